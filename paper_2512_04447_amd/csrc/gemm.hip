// Complex Gram and rotation GEMMs on CDNA4 MFMA (task (2) of the SCF task
// list: the dense products that form the LOBPCG subspace matrices H and S,
// and the rotation of the block by the Ritz coefficients).
//
// Complex products use four real MFMAs per 16x16x4 step on the real and
// imaginary parts (no Gauss trick, which loses accuracy).  Operand layout of
// v_mfma_{f64,f32}_16x16x4 (measured on gfx950): lane l holds A[l%16][l/16]
// and B[l/16][l%16]; the 16x16 result sits in 4 accumulators per lane,
// column l%16, row 4*(l/16)+v for f32 but row l/16+4*v for f64.
#include "gemm.hpp"

namespace ks {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = d4;
  __device__ static inline acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
  using acc = f4;
  __device__ static inline acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int TILE = 64;  // output tile edge per workgroup
constexpr int KC = 16;    // K chunk staged in LDS (small GEMMs)
constexpr int PAD = KC + 1;
constexpr int ROT_KC = 16;  // K chunk of the rotation
// K chunk of the Gram: 16 (FP64) or 32 (FP32) points, so that one chunk of
// the three operand panels stays near 52 KB of LDS either way.
template <typename T> constexpr int gram_kc() { return sizeof(T) == 4 ? 32 : 16; }

// Column c of a three-segment block list (segments of nb columns each).
// Two compares and selects between the three base pointers: a division and
// an indexed read of the pointer array cost a dependent load from the
// argument segment on every call.
template <typename T2>
__device__ inline const T2* seg_col(const BlockList<T2>& b, int c) {
  const int s = (c >= b.nb ? 1 : 0) + (c >= 2 * b.nb ? 1 : 0);
  const T2* base = s == 0 ? b.p[0] : (s == 1 ? b.p[1] : b.p[2]);
  return base + (int64_t)(c - s * b.nb) * b.ld;
}

// ---------------------------------------------------------------- Gram
// v when c, else zero, selected per component (a select between two
// vector structs was lowered through scratch memory)
template <typename T2> __device__ __forceinline__ T2 keep_if(bool c, T2 v) {
  using S = decltype(v.x);
  return cmake<T2>(c ? v.x : S(0), c ? v.y : S(0));
}

// For upper tile (ti, tj) and K split `sp`: S_tile = A_I^H B1_J and, when
// TWO, H_tile = A_I^H B2_J.  Partials (FP64) go to part[(sp*ntu + t)*4096 +
// i*64 + j] (row-major within the tile).
// Loads of one K chunk into registers: point kb + lk of the EPT columns
// qa[q], qb[q], qb2[q] of each operand.  Plain functions rather than
// lambdas: arrays captured by reference in a lambda were kept in private
// memory.  The loads are unconditional, from valid columns at a point
// clamped to k1 - 1 (k1 > kb).  Nothing is zeroed here (a select on the
// loaded value would wait for the load at once): the caller zeroes the A
// values of a point past k1 when it stores them to LDS, and the values of
// a clamped column only reach Gram entries that are not stored.
template <bool TWO, int EPT, typename T2>
__device__ __forceinline__ void gram_fetch(T2 (&ra)[EPT], T2 (&rb)[EPT], T2 (&rb2)[TWO ? EPT : 1],
                                           const T2* const (&qa)[EPT], const T2* const (&qb)[EPT],
                                           const T2* const (&qb2)[EPT], int64_t kb, int lk, int64_t k1) {
  const int64_t k = kb + lk;
  const int64_t e = k < k1 ? k : k1 - 1;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    ra[q] = gload(qa[q] + e);
    rb[q] = gload(qb[q] + e);
    if constexpr (TWO) rb2[q] = gload(qb2[q] + e);
  }
}

// FP32 accumulators into the FP64 sums, then cleared.
template <bool TWO, int WN, typename A>
__device__ __forceinline__ void gram_flush(A (&sr)[2][WN], A (&si)[2][WN], A (&hr)[2][WN], A (&hi)[2][WN],
                                           double (&dsr)[2][WN][4], double (&dsi)[2][WN][4],
                                           double (&dhr)[2][WN][4], double (&dhi)[2][WN][4]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dsr[a][b][v] += (double)sr[a][b][v];
        dsi[a][b][v] += (double)si[a][b][v];
        sr[a][b][v] = si[a][b][v] = 0.0f;
        if constexpr (TWO) {
          dhr[a][b][v] += (double)hr[a][b][v];
          dhi[a][b][v] += (double)hi[a][b][v];
          hr[a][b][v] = hi[a][b][v] = 0.0f;
        }
      }
}

// Waves per tile in a 2 x WJ grid.  FP32: WJ = 4 (512 threads), a wave owns
// a 32 x 16 sub-tile, which keeps the accumulators and the FP64 shadow sums
// small enough for three waves per SIMD.  FP64: WJ = 2 (256 threads), a wave
// owns 32 x 32 (measured faster for FP64 at both cell sizes).
template <typename T> constexpr int gram_wj() { return sizeof(T) == 4 ? 4 : 2; }
template <typename T> constexpr int gram_threads() { return 128 * gram_wj<T>(); }
// FP64: ask for two resident blocks per CU (two waves per SIMD)
template <typename T> constexpr int gram_min_blocks() { return sizeof(T) == 8 ? 2 : 1; }

template <typename T, bool TWO>
__global__ void __launch_bounds__(gram_threads<T>(), gram_min_blocks<T>())
k_gram(BlockList<c2<T>> A, BlockList<c2<T>> B1, BlockList<c2<T>> B2, int m, int64_t K, int64_t kper,
       int ntile, int ntu, int full, double2* __restrict__ partS, double2* __restrict__ partH) {
  using T2 = c2<T>;
  using M = Mfma<T>;
  constexpr int GKC = gram_kc<T>();
  constexpr int GPAD = GKC + 1;
  constexpr int WJ = gram_wj<T>();
  constexpr int WN = TILE / WJ / 16;          // 16-column MFMA tiles per wave
  constexpr int EPT = TILE * GKC / gram_threads<T>();  // columns per loader thread and operand
  __shared__ T2 As[TILE][GPAD];
  __shared__ T2 Bs[TILE][GPAD];
  __shared__ T2 B2s[TWO ? TILE : 1][GPAD];
  // tile index -> (ti, tj): upper tiles ti <= tj, or every tile when full
  int t = blockIdx.x;
  int ti = 0;
  if (full) {
    ti = t / ntile;
    t -= ti * ntile;
  } else {
    while (t >= ntile - ti) { t -= ntile - ti; ++ti; }
  }
  const int tj = full ? t : ti + t;
  const int sp = blockIdx.y;
  const int64_t k0 = (int64_t)sp * kper;
  const int64_t k1 = min(K, k0 + kper);
  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int wi = wave / WJ, wj = wave % WJ;
  // A Hermitian Gram's diagonal tile needs its upper half only: the waves
  // of rows 32..63 and columns 0..31 (strictly below the diagonal) issue no
  // MFMA, and the reduction takes those entries from their mirrors.
  const bool lower_skip = !full && ti == tj && wi == 1 && wj * WN * 16 < 32;
  const bool wact = ti * TILE + wi * 32 < m && tj * TILE + wj * WN * 16 < m && !lower_skip;
  typename M::acc sr[2][WN], si[2][WN], hr[2][WN], hi[2][WN];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) sr[a][b][v] = si[a][b][v] = hr[a][b][v] = hi[a][b][v] = T(0);
  // loader: thread -> point lk of the chunk in the columns lc + CST q
  // (q < EPT): lanes run along the points of a column, so the loads are
  // coalesced and the LDS stores free of bank conflicts
  constexpr int CST = gram_threads<T>() / GKC;
  static_assert(CST * EPT == TILE, "loader columns cover the tile");
  const int lk = threadIdx.x % GKC;
  const int lc = threadIdx.x / GKC;
  const T2 z = cmake<T2>(T(0), T(0));
  const T2* pb0 = seg_col(A, 0);  // a valid column for loads that are discarded
  const T2* qa[EPT];
  const T2* qb[EPT];
  const T2* qb2[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int ca = ti * TILE + lc + CST * q, cb = tj * TILE + lc + CST * q;
    qa[q] = ca < m ? seg_col(A, ca) : pb0;
    qb[q] = cb < m ? seg_col(B1, cb) : pb0;
    qb2[q] = (TWO && cb < m) ? seg_col(B2, cb) : pb0;
  }
  // FP32 products accumulate in FP32 over KFLUSH points, then in FP64.
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int KFLUSH = 256;
  double dsr[F32 ? 2 : 1][WN][4], dsi[F32 ? 2 : 1][WN][4], dhr[F32 ? 2 : 1][WN][4], dhi[F32 ? 2 : 1][WN][4];
  if constexpr (F32) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < WN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) dsr[a][b][v] = dsi[a][b][v] = dhr[a][b][v] = dhi[a][b][v] = 0.0;
  }
  // FP32: register stage of the next chunk, whose global loads are in flight
  // while the current chunk is multiplied out of LDS.  FP64 loads each chunk
  // just before storing it (measured faster: the FP64 kernel is limited by
  // its accumulator registers, not by load latency).
  constexpr bool PREFETCH = F32;
  constexpr int NR = PREFETCH ? EPT : 1;
  T2 ra[NR], rb[NR], rb2[TWO ? NR : 1];
  if constexpr (PREFETCH) {
    if (k0 < k1) gram_fetch<TWO>(ra, rb, rb2, qa, qb, qb2, k0, lk, k1);
  }
  for (int64_t kb = k0; kb < k1; kb += GKC) {
    if constexpr (PREFETCH) {
      const bool ok = kb + lk < k1;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        As[lc + CST * q][lk] = keep_if(ok, ra[q]);
        Bs[lc + CST * q][lk] = rb[q];
        if (TWO) B2s[lc + CST * q][lk] = rb2[q];
      }
    } else {
      // FP64: all loads of the chunk issued before the first is used, then
      // stored; the A values of a point past k1 zeroed
      T2 la[EPT], lb[EPT], lb2[TWO ? EPT : 1];
      gram_fetch<TWO>(la, lb, lb2, qa, qb, qb2, kb, lk, k1);
      const bool ok = kb + lk < k1;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        As[lc + CST * q][lk] = keep_if(ok, la[q]);
        Bs[lc + CST * q][lk] = lb[q];
        if (TWO) B2s[lc + CST * q][lk] = lb2[q];
      }
    }
    __syncthreads();
    if constexpr (PREFETCH) {
      if (kb + GKC < k1) gram_fetch<TWO>(ra, rb, rb2, qa, qb, qb2, kb + GKC, lk, k1);
    }
    if constexpr (F32) {
      if (kb > k0 && ((kb - k0) % KFLUSH) == 0) gram_flush<TWO>(sr, si, hr, hi, dsr, dsi, dhr, dhi);
    }
    // a wave whose rows or columns all lie past m has only padding to
    // compute: it loads and waits with the others but issues no MFMA, and
    // the co-resident workgroup's wave on its SIMD takes the matrix core
    if (wact)
#pragma unroll
    for (int kk = 0; kk < GKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      T2 a[2], b[WN], b2[WN];
#pragma unroll
      for (int u = 0; u < 2; ++u) a[u] = As[wi * 32 + u * 16 + (lane & 15)][kr];
#pragma unroll
      for (int w = 0; w < WN; ++w) {
        b[w] = Bs[wj * WN * 16 + w * 16 + (lane & 15)][kr];
        if (TWO) b2[w] = B2s[wj * WN * 16 + w * 16 + (lane & 15)][kr];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < WN; ++w) {
          // conj(a) * b: re = ar br + ai bi, im = ar bi - ai br
          sr[u][w] = M::run(a[u].x, b[w].x, sr[u][w]);
          sr[u][w] = M::run(a[u].y, b[w].y, sr[u][w]);
          si[u][w] = M::run(a[u].x, b[w].y, si[u][w]);
          si[u][w] = M::run(-a[u].y, b[w].x, si[u][w]);
          if (TWO) {
            hr[u][w] = M::run(a[u].x, b2[w].x, hr[u][w]);
            hr[u][w] = M::run(a[u].y, b2[w].y, hr[u][w]);
            hi[u][w] = M::run(a[u].x, b2[w].y, hi[u][w]);
            hi[u][w] = M::run(-a[u].y, b2[w].x, hi[u][w]);
          }
        }
    }
    __syncthreads();
  }
  if constexpr (F32) gram_flush<TWO>(sr, si, hr, hi, dsr, dsi, dhr, dhi);
  const int64_t base = ((int64_t)sp * ntu + blockIdx.x) * (TILE * TILE);
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < WN; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wi * 32 + u * 16 + M::row(lane, v);
        const int j = wj * WN * 16 + w * 16 + (lane & 15);
        if constexpr (F32) {
          partS[base + i * TILE + j] = make_double2(dsr[u][w][v], dsi[u][w][v]);
          if (TWO) partH[base + i * TILE + j] = make_double2(dhr[u][w][v], dhi[u][w][v]);
        } else {
          partS[base + i * TILE + j] = make_double2((double)sr[u][w][v], (double)si[u][w][v]);
          if (TWO) partH[base + i * TILE + j] = make_double2((double)hr[u][w][v], (double)hi[u][w][v]);
        }
      }
}

// Sum the K splits in order and write the Hermitian m x m result
// (column-major, ldo).  Diagonal tiles are Hermitised, (G + G^H)/2, within
// their 32 x 32 diagonal blocks.
__global__ void __launch_bounds__(256)
k_gram_reduce(const double2* __restrict__ part, int nsplit, int ntile, int ntu, int m, int full,
              double2* __restrict__ out, int ldo) {
  int t = blockIdx.x;
  int ti = 0;
  if (full) {
    ti = t / ntile;
    t -= ti * ntile;
  } else {
    while (t >= ntile - ti) { t -= ntile - ti; ++ti; }
  }
  const int tj = full ? t : ti + t;
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < TILE * TILE; e += gridDim.y * blockDim.x) {
    const int i = e / TILE, j = e - i * TILE;
    const int gi = ti * TILE + i, gj = tj * TILE + j;
    if (gi >= m || gj >= m) continue;
    if (full) {
      double2 s = make_double2(0.0, 0.0);
      for (int sp = 0; sp < nsplit; ++sp) {
        const double2 v = part[((int64_t)sp * ntu + blockIdx.x) * (TILE * TILE) + e];
        s.x += v.x;
        s.y += v.y;
      }
      out[gi + (int64_t)gj * ldo] = s;
      continue;
    }
    if (ti == tj && j < i) continue;  // handled by its mirror
    double2 s = make_double2(0.0, 0.0);
    for (int sp = 0; sp < nsplit; ++sp) {
      const double2 v = part[((int64_t)sp * ntu + blockIdx.x) * (TILE * TILE) + e];
      s.x += v.x;
      s.y += v.y;
    }
    // a diagonal tile: the two triangles averaged where both were computed
    // (within the 32 x 32 diagonal blocks); rows 32..63 of columns 0..31
    // were not (k_gram skips them), their mirrors stand alone
    if (ti == tj && !(i < 32 && j >= 32)) {
      double2 s2 = make_double2(0.0, 0.0);
      for (int sp = 0; sp < nsplit; ++sp) {
        const double2 v = part[((int64_t)sp * ntu + blockIdx.x) * (TILE * TILE) + j * TILE + i];
        s2.x += v.x;
        s2.y += v.y;
      }
      s.x = 0.5 * (s.x + s2.x);
      s.y = 0.5 * (s.y - s2.y);
      if (i == j) s.y = 0.0;
    }
    out[gi + (int64_t)gj * ldo] = s;
    out[gj + (int64_t)gi * ldo] = make_double2(s.x, -s.y);
  }
}

// K splits: each workgroup sums one tile over one K range into FP64
// partials, reduced afterwards.  The split count makes the number of
// workgroups fill whole rounds of the device's resident slots (workgroups
// are of equal length, so a last round that is nearly empty costs as much
// as a full one): the count minimises rounds / splits, a smaller count
// winning ties within 2%, with at least 512 points per split and partials
// under GRAM_PART_BYTES.
constexpr int64_t GRAM_PART_BYTES = 1ll << 30;

GramShape gram_shape(int ntile, int64_t K, bool full, int slots) {
  GramShape g;
  g.ntile = ntile;
  g.ntu = full ? ntile * ntile : ntile * (ntile + 1) / 2;
  if (slots <= 0) slots = 1024;
  const int64_t ns_k = std::max<int64_t>(1, K / 512);
  const int64_t ns_mem = std::max<int64_t>(1, GRAM_PART_BYTES / ((int64_t)g.ntu * TILE * TILE * 16 * 2));
  const int64_t nsmax = std::min<int64_t>(std::min(ns_k, ns_mem), 4096);
  int64_t best = 1;
  double bestc = 1e300;
  for (int64_t ns = 1; ns <= nsmax; ++ns) {
    const double rounds = (double)ceil_div((int64_t)g.ntu * ns, slots);
    const double cost = rounds / (double)ns;
    if (cost < 0.98 * bestc) {
      bestc = cost;
      best = ns;
    }
  }
  g.kper = ceil_div(ceil_div(K, best), 32) * 32;  // a multiple of either Gram chunk
  g.nsplit = (int)ceil_div(K, g.kper);
  return g;
}

// Resident workgroups of one Gram kernel on the current device.
template <typename T, bool TWO> static int gram_slots() {
  static int cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] > 0) return cache[dev];
  int per = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_gram<T, TWO>),
                                                   gram_threads<T>(), 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  cache[dev] = std::max(1, per) * std::max(1, cus);
  return cache[dev];
}

size_t gram_work_bytes(int m, int64_t K) {
  const int slots[4] = {gram_slots<double, true>(), gram_slots<double, false>(), gram_slots<float, true>(),
                        gram_slots<float, false>()};
  size_t mx = 0;
  const int nt = (int)ceil_div(std::max(m, 1), TILE);
  for (int t = 1; t <= nt; ++t)
    for (int f = 0; f < 2; ++f)
      for (int v = 0; v < 4; ++v) {
        const GramShape g = gram_shape(t, K, f == 1, slots[v]);
        mx = std::max(mx, (size_t)g.nsplit * g.ntu * TILE * TILE * sizeof(double2) * 2);
      }
  return mx;
}

template <typename T>
static int gram_impl(const BlockList<c2<T>>& A, const BlockList<c2<T>>& B1, const BlockList<c2<T>>* B2, int m,
                     int64_t K, bool full, double2* S, int lds_, double2* H, int ldh, void* work, hipStream_t s) {
  if (m <= 0) return 0;
  const GramShape g = gram_shape((int)ceil_div(m, TILE), K, full, B2 ? gram_slots<T, true>() : gram_slots<T, false>());
  double2* partS = static_cast<double2*>(work);
  double2* partH = partS + (size_t)g.nsplit * g.ntu * TILE * TILE;
  dim3 grid(g.ntu, g.nsplit);
  const int fl = full ? 1 : 0;
  TimerScope ts(KF_GRAM, s);
  if (B2)
    hipLaunchKernelGGL((k_gram<T, true>), grid, dim3(gram_threads<T>()), 0, s, A, B1, *B2, m, K, g.kper, g.ntile, g.ntu, fl, partS,
                       partH);
  else
    hipLaunchKernelGGL((k_gram<T, false>), grid, dim3(gram_threads<T>()), 0, s, A, B1, B1, m, K, g.kper, g.ntile, g.ntu, fl, partS,
                       partH);
  KS_LAUNCH_CHECK("gram");
  hipLaunchKernelGGL(k_gram_reduce, dim3(g.ntu, 16), dim3(256), 0, s, partS, g.nsplit, g.ntile, g.ntu, m, fl, S, lds_);
  KS_LAUNCH_CHECK("gram_reduce");
  if (B2) {
    hipLaunchKernelGGL(k_gram_reduce, dim3(g.ntu, 16), dim3(256), 0, s, partH, g.nsplit, g.ntile, g.ntu, m, fl, H, ldh);
    KS_LAUNCH_CHECK("gram_reduce");
  }
  return 0;
}

template <typename T>
int gram(const BlockList<c2<T>>& A, const BlockList<c2<T>>& B1, const BlockList<c2<T>>* B2, int m, int64_t K,
         double2* S, int lds_, double2* H, int ldh, void* work, hipStream_t s) {
  return gram_impl<T>(A, B1, B2, m, K, false, S, lds_, H, ldh, work, s);
}

template <typename T>
int gram_general(const BlockList<c2<T>>& A, const BlockList<c2<T>>& B, int m, int64_t K, double2* G, int ldg,
                 void* work, hipStream_t s) {
  return gram_impl<T>(A, B, nullptr, m, K, true, G, ldg, nullptr, 0, work, s);
}

template int gram_general<double>(const BlockList<double2>&, const BlockList<double2>&, int, int64_t, double2*, int,
                                  void*, hipStream_t);
template int gram_general<float>(const BlockList<float2>&, const BlockList<float2>&, int, int64_t, double2*, int,
                                 void*, hipStream_t);

// ---------------------------------------------------------------- rotation
// Y = V C for a block list V (Ng x m) and C (m x ncol, column-major, ldc in
// the block precision).  Computed as Y^T = C^T V^T so that the accumulator
// layout stores 16 consecutive grid points per band (coalesced).  When Yp
// is given, the sum over columns [pstart, m) is stored to Yp first, then the
// columns [0, pstart) are added and the total stored to Y.
// With upper (C upper triangular: C[i][band] = 0 for i > band, as for the
// Cholesky-QR coefficients D L^-H) a band tile [b0, b0 + 64) stops at
// column b0 + 64 of V, and each 16-band MFMA sub-tile stops issuing at its
// own last band: the skipped terms are exact zeros, the result the same.
// With Yadd (no Yp), Y = Yadd + V C: each element of Yadd is read by the
// thread that writes the same element of Y, so Yadd may be Y.
//
// A workgroup takes `rtiles` consecutive 64-point row tiles of one band
// tile (a one-dimensional grid of ceil(row tiles / rtiles) x band tiles).
// Its chunk loads run one chunk ahead across the tiles (and the two sums
// of Yp), so the load latency at the start of a tile and the stores at its
// end overlap the products of the neighbouring chunks.
template <typename T, int RKC>
__global__ void __launch_bounds__(256, 3)
k_rotate(BlockList<c2<T>> V, int m, int pstart, const c2<T>* __restrict__ C, int ldc, int ncol, int64_t Ng,
         c2<T>* Y, c2<T>* __restrict__ Yp, int64_t ldy, int upper, const c2<T>* Yadd, int rtiles) {
  using T2 = c2<T>;
  using M = Mfma<T>;
  constexpr int EP = RKC / 4;       // V and C values per loader thread
  __shared__ T2 Vs[RKC][TILE + 1];  // [i][r]
  __shared__ T2 Cs[TILE][RKC + 1];  // [band][i]
  const int64_t ntr = (Ng + TILE - 1) / TILE;
  // Workgroup order: the workgroups one XCD receives in a row take the band
  // tiles of the same row tiles, which then read the same V chunks at about
  // the same time, once from HBM for the whole XCD.
  const int nbt = (ncol + TILE - 1) / TILE;
  const int64_t g = xcd_order(blockIdx.x, gridDim.x);
  const int64_t t_first = (g / nbt) * rtiles;
  const int nt = (int)min((int64_t)rtiles, ntr - t_first);
  const int b0 = (int)(g % nbt) * TILE;
  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int wb = wave >> 1, wr = wave & 1;  // wave's band half, row half
  const bool wact = b0 + wb * 32 < ncol;
  // sums: 0 = [pstart, m) into Yp then 1 = [0, pstart) into Y when Yp is
  // given; else one sum over [0, m) (or [0, b0 + 64) when upper)
  const int npass = Yp ? 2 : 1;
  auto lo_of = [&](int p) { return (Yp && p == 0) ? pstart : 0; };
  auto hi_of = [&](int p) { return Yp ? (p == 0 ? m : pstart) : (upper ? min(m, b0 + TILE) : m); };
  // last chunk start (exclusive bound) of each 16-band sub-tile u under upper
  const int ulim0 = upper ? b0 + wb * 32 + 16 : m, ulim1 = upper ? b0 + wb * 32 + 32 : m;
  typename M::acc dr[2][2], di[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) dr[a][b][v] = di[a][b][v] = T(0);
  // loaders, lanes along the contiguous index of each operand (coalesced
  // loads, LDS stores without bank conflicts): V row vr of the columns
  // vi + 4 e; C coefficient ci of the bands cb + (256 / RKC) e, e < EP
  const int vr = threadIdx.x % TILE, vi = threadIdx.x / TILE;
  const int ci = threadIdx.x % RKC, cb = threadIdx.x / RKC;
  constexpr int CBS = 256 / RKC;  // band stride between a thread's coefficients
  // register stage of the next chunk (its loads overlap this chunk's MFMAs)
  T2 vv[EP], qq[EP];
  // Unconditional global loads from indices clamped into range (column 0,
  // row Ng - 1, band 0, coefficient hi - 1); a guarded load through a
  // pointer selected against null became a flat load, whose wait also held
  // up the LDS reads of the current chunk.  Only the coefficients past hi
  // are zeroed, when they are stored to LDS (not at the load, which would
  // wait for it there): a clamped V column then meets a zero coefficient,
  // and clamped rows or bands only reach outputs that are not stored.
  const T2* ccol[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int band = b0 + cb + CBS * e;
    ccol[e] = C + (int64_t)(band < ncol ? band : 0) * ldc;
  }
  const int64_t rl = Ng - 1;
  // fetch cursor (tile ft, sum fp, chunk fc): always the chunk after the
  // one being multiplied, in the same order as the loops below
  int ft = 0, fp = 0, fc = lo_of(0);
  auto settle = [&]() {
    while (ft < nt && fc >= hi_of(fp)) {
      if (++fp == npass) {
        fp = 0;
        ++ft;
      }
      fc = lo_of(fp);
    }
  };
  auto fetch = [&]() {
    const int hi = hi_of(fp);
    const int64_t r = min((t_first + ft) * TILE + vr, rl);
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      const int c_ = fc + vi + 4 * e;
      vv[e] = gload(seg_col(V, c_ < hi ? c_ : 0) + r);
    }
    const int i_ = min(fc + ci, hi - 1);
#pragma unroll
    for (int e = 0; e < EP; ++e) qq[e] = gload(ccol[e] + i_);
  };
  settle();
  if (ft < nt) fetch();
  for (int t = 0; t < nt; ++t) {
    const int64_t r0 = (t_first + t) * TILE;
    for (int pass = 0; pass < npass; ++pass) {
      const int lo = lo_of(pass), hi = hi_of(pass);
      for (int c0 = lo; c0 < hi; c0 += RKC) {
#pragma unroll
        for (int e = 0; e < EP; ++e) {
          Vs[vi + 4 * e][vr] = vv[e];
          Cs[cb + CBS * e][ci] = keep_if(c0 + ci < hi, qq[e]);
        }
        __syncthreads();
        fc += RKC;
        settle();
        if (ft < nt) fetch();
        // a wave whose 32 bands all lie past ncol issues no MFMA (padding)
        const bool on0 = wact && c0 < ulim0, on1 = wact && c0 < ulim1;
#pragma unroll
        for (int kk = 0; kk < RKC; kk += 4) {
          const int kr = kk + (lane >> 4);
          T2 a[2], b[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            a[u] = Cs[wb * 32 + u * 16 + (lane & 15)][kr];  // A = C^T: [band][i]
            b[u] = Vs[kr][wr * 32 + u * 16 + (lane & 15)];  // B = V^T: [i][r]
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (!(u == 0 ? on0 : on1)) continue;
#pragma unroll
            for (int w = 0; w < 2; ++w) {
              // c * v: re = cr vr - ci vi, im = cr vi + ci vr
              dr[u][w] = M::run(a[u].x, b[w].x, dr[u][w]);
              dr[u][w] = M::run(-a[u].y, b[w].y, dr[u][w]);
              di[u][w] = M::run(a[u].x, b[w].y, di[u][w]);
              di[u][w] = M::run(a[u].y, b[w].x, di[u][w]);
            }
          }
        }
        __syncthreads();
      }
      T2* out = (Yp && pass == 0) ? Yp : Y;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int band = b0 + wb * 32 + u * 16 + M::row(lane, v);
            const int64_t r = r0 + wr * 32 + w * 16 + (lane & 15);
            if (band < ncol && r < Ng) {
              T2 o = cmake<T2>(dr[u][w][v], di[u][w][v]);
              if (Yadd != nullptr && out == Y) {
                const T2 a = Yadd[(int64_t)band * ldy + r];
                o = cmake<T2>(a.x + o.x, a.y + o.y);
              }
              out[(int64_t)band * ldy + r] = o;
            }
          }
      // a new tile starts from zero; Y of a tile with Yp adds the second
      // sum to the first (the accumulators carry over between the sums)
      if (pass == npass - 1) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) dr[a][b][v] = di[a][b][v] = T(0);
      }
    }
  }
}

template <typename T>
int rotate(const BlockList<c2<T>>& V, int m, int pstart, const c2<T>* C, int ldc, int ncol, int64_t Ng,
           c2<T>* Y, c2<T>* Yp, int64_t ldy, hipStream_t s, bool upper, const c2<T>* Yadd) {
  if (ncol <= 0) return 0;
  // row tiles per workgroup: up to 8 while the grid keeps about eight
  // workgroups per resident slot (three per CU on 256 CUs)
  const int64_t ntr = ceil_div(Ng, TILE), nbt = ceil_div(ncol, TILE);
  const int rt = (int)std::max<int64_t>(1, std::min<int64_t>(8, ntr * nbt / (8 * 768)));
  dim3 grid((unsigned)(ceil_div(ntr, rt) * nbt));
  TimerScope ts(KF_ROTATE, s);
  hipLaunchKernelGGL((k_rotate<T, ROT_KC>), grid, dim3(256), 0, s, V, m, pstart, C, ldc, ncol, Ng, Y, Yp, ldy,
                     (upper && Yp == nullptr) ? 1 : 0, Yp == nullptr ? Yadd : nullptr, rt);
  KS_LAUNCH_CHECK("rotate");
  return 0;
}

// ---------------------------------------------------------------- zgemm
// C = alpha op(A) op(B) + beta C, FP64 complex, column-major; op = 'N' or 'C'
// (conjugate transpose); alpha and beta real.  For the small subspace
// matrices of the dense solver.
template <bool CA, bool CB>
__global__ void __launch_bounds__(256)
k_zgemm(int M, int N, int K, double alpha, const double2* __restrict__ A, int lda,
        const double2* __restrict__ B, int ldb, double beta, double2* __restrict__ C, int ldc) {
  using Mf = Mfma<double>;
  __shared__ double2 As[KC][TILE + 1];  // [k][i]
  __shared__ double2 Bs[TILE][PAD];     // [j][k]
  const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) cr[a][b][v] = ci[a][b][v] = 0.0;
  const double2 z = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    // the A tile op(A)[i][k] and the B tile op(B)[k][j], four elements of
    // each per thread with all eight loads in flight: unconditional, from
    // indices clamped into range, zeroed afterwards (guarded loads went one
    // at a time)
    static_assert(KC * TILE == 4 * 256, "four elements of each tile per thread");
    double2 av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      int i, k;
      if (!CA) { i = e % TILE; k = e / TILE; } else { k = e % KC; i = e / KC; }
      const int gi = min(i0 + i, M - 1), gk = min(k0 + k, K - 1);
      av[u] = !CA ? A[gi + (int64_t)gk * lda] : A[gk + (int64_t)gi * lda];
      int j, kb;
      if (!CB) { kb = e % KC; j = e / KC; } else { j = e % TILE; kb = e / TILE; }
      const int gj = min(j0 + j, N - 1), gkb = min(k0 + kb, K - 1);
      bv[u] = !CB ? B[gkb + (int64_t)gj * ldb] : B[gj + (int64_t)gkb * ldb];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      int i, k;
      if (!CA) { i = e % TILE; k = e / TILE; } else { k = e % KC; i = e / KC; }
      const bool oka = i0 + i < M && k0 + k < K;
      As[k][i] = make_double2(oka ? av[u].x : 0.0, oka ? (CA ? -av[u].y : av[u].y) : 0.0);
      int j, kb;
      if (!CB) { kb = e % KC; j = e / KC; } else { j = e % TILE; kb = e / TILE; }
      const bool okb = j0 + j < N && k0 + kb < K;
      Bs[j][kb] = make_double2(okb ? bv[u].x : 0.0, okb ? (CB ? -bv[u].y : bv[u].y) : 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double2 a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = As[kr][wi * 32 + u * 16 + (lane & 15)];
        b[u] = Bs[wj * 32 + u * 16 + (lane & 15)][kr];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          cr[u][w] = Mf::run(a[u].x, b[w].x, cr[u][w]);
          cr[u][w] = Mf::run(-a[u].y, b[w].y, cr[u][w]);
          ci[u][w] = Mf::run(a[u].x, b[w].y, ci[u][w]);
          ci[u][w] = Mf::run(a[u].y, b[w].x, ci[u][w]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wi * 32 + u * 16 + Mf::row(lane, v);
        const int gj = j0 + wj * 32 + w * 16 + (lane & 15);
        if (gi < M && gj < N) {
          double2* c = C + gi + (int64_t)gj * ldc;
          double2 o = make_double2(alpha * cr[u][w][v], alpha * ci[u][w][v]);
          if (beta != 0.0) {
            o.x += beta * c->x;
            o.y += beta * c->y;
          }
          *c = o;
        }
      }
}

int zgemm(char ta, char tb, int M, int N, int K, double alpha, const double2* A, int lda, const double2* B,
          int ldb, double beta, double2* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  dim3 grid((unsigned)ceil_div(M, TILE), (unsigned)ceil_div(N, TILE));
  const bool ca = ta == 'C', cb = tb == 'C';
  TimerScope ts(KF_ZGEMM, s);
  if (!ca && !cb)
    hipLaunchKernelGGL((k_zgemm<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (ca && !cb)
    hipLaunchKernelGGL((k_zgemm<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!ca && cb)
    hipLaunchKernelGGL((k_zgemm<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL((k_zgemm<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  KS_LAUNCH_CHECK("zgemm");
  return 0;
}

template int gram<double>(const BlockList<double2>&, const BlockList<double2>&, const BlockList<double2>*, int,
                          int64_t, double2*, int, double2*, int, void*, hipStream_t);
template int gram<float>(const BlockList<float2>&, const BlockList<float2>&, const BlockList<float2>*, int,
                         int64_t, double2*, int, double2*, int, void*, hipStream_t);
template int rotate<double>(const BlockList<double2>&, int, int, const double2*, int, int, int64_t, double2*,
                            double2*, int64_t, hipStream_t, bool, const double2*);
template int rotate<float>(const BlockList<float2>&, int, int, const float2*, int, int, int64_t, float2*, float2*,
                           int64_t, hipStream_t, bool, const float2*);

}  // namespace ks
