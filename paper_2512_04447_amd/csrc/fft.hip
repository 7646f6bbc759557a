// Batched 3D FFT Hamiltonian application and Teter-Payne-Allan
// preconditioner for gfx950.
//
// The paper applies the kinetic term through FFTs over all orbitals at once
// (task (1) of the SCF task list; the FFT figure shows batching is what makes
// GPUs win).  Here a 3D transform of one band is split into three passes
// over HBM, each staging tiles in LDS:
//   pass A: per (band, x-plane): z- then y-transforms of the n1 x n2 plane;
//   pass B: per (band, y, z-chunk): x-transform of an x-pencil tile, a
//           spectral multiply, then the inverse x-transform;
//   pass C: per (band, x-plane): inverse y- and z-transforms, 1/Ng, and an
//           epilogue (local potential and nonlocal scatter for H, lock mask
//           for the preconditioner).
// Each 1D transform is a mixed-radix (16, 8, 7, 6, 5, 4, 3, 2) Stockham autosort FFT
// done in place in LDS: a stage reads its butterfly inputs into registers,
// barriers, then writes the outputs to their autosorted positions.  The
// inverse transform is conj(FFT(conj(.))).
#include <cmath>

#include "ks_plan.hpp"

namespace ks {

// ---------------------------------------------------------------- radices
template <typename T2> __device__ inline T2 mul_minus_i(T2 a) { return cmake<T2>(a.y, -a.x); }

template <int R, typename T2> struct Dft;

template <typename T2> struct Dft<2, T2> {
  __device__ static void run(T2* a) {
    T2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <typename T2> struct Dft<3, T2> {
  __device__ static void run(T2* a) {
    using T = decltype(a[0].x);
    const T s1 = T(-0.86602540378443864676);  // sin(-2 pi / 3)
    T2 t1 = cadd(a[1], a[2]);
    T2 t2 = csub(a[1], a[2]);
    T2 y0 = cadd(a[0], t1);
    T2 m1 = csub(a[0], cscale(t1, T(0.5)));
    T2 m2 = cmake<T2>(-s1 * t2.y, s1 * t2.x);  // i * s1 * t2
    a[0] = y0;
    a[1] = cadd(m1, m2);
    a[2] = csub(m1, m2);
  }
};

template <typename T2> struct Dft<4, T2> {
  __device__ static void run(T2* a) {
    T2 t0 = cadd(a[0], a[2]);
    T2 t1 = csub(a[0], a[2]);
    T2 t2 = cadd(a[1], a[3]);
    T2 t3 = mul_minus_i(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

// Odd radix by symmetric pairs: with s_q = a_q + a_{R-q}, d_q = a_q - a_{R-q},
// y_k = a_0 + sum_q s_q cos(2 pi q k/R) - i sum_q d_q sin(2 pi q k/R) and
// y_{R-k} the same with +i.
template <int R> struct OddRoots;
template <> struct OddRoots<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                  -0.80901699437494742410, 0.30901699437494742410};
  static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                  -0.58778525229247312917, -0.95105651629515357212};
};
template <> struct OddRoots<7> {
  static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                  -0.90096886790241912624, -0.90096886790241912624,
                                  -0.22252093395631440429, 0.62348980185873353053};
  static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                  0.43388373911755812048, -0.43388373911755812048,
                                  -0.97492791218182360702, -0.78183148246802980871};
};

template <int R, typename T2> struct DftOdd {
  __device__ static void run(T2* a) {
    using T = decltype(a[0].x);
    constexpr int H = (R - 1) / 2;
    T2 sq[H], dq[H];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      sq[q - 1] = cadd(a[q], a[R - q]);
      dq[q - 1] = csub(a[q], a[R - q]);
    }
    T2 y0 = a[0];
#pragma unroll
    for (int q = 0; q < H; ++q) y0 = cadd(y0, sq[q]);
    T2 out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      T2 A = a[0];
      T2 B = cmake<T2>(T(0), T(0));
#pragma unroll
      for (int q = 1; q <= H; ++q) {
        const int idx = (q * k) % R;
        const T c = T(OddRoots<R>::c[idx]);
        const T s = T(OddRoots<R>::s[idx]);
        A = cadd(A, cscale(sq[q - 1], c));
        B = cadd(B, cscale(dq[q - 1], s));
      }
      // y_k = A - i B, y_{R-k} = A + i B
      out[k] = cmake<T2>(A.x + B.y, A.y - B.x);
      out[R - k] = cmake<T2>(A.x - B.y, A.y + B.x);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = out[k];
  }
};
template <typename T2> struct Dft<5, T2> : DftOdd<5, T2> {};
template <typename T2> struct Dft<7, T2> : DftOdd<7, T2> {};

// exp(-2 pi i m / N) = (c[m], -s[m]) for the composite radices below, from
// the closed forms of the angles (multiples of pi/3 and pi/8).
template <int N> struct TwN;
#define KS_R2 0.70710678118654752440
#define KS_R3 0.86602540378443864676
#define KS_C8 0.92387953251128675613
#define KS_S8 0.38268343236508977173
template <> struct TwN<6> {
  static constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
  static constexpr double s[6] = {0.0, KS_R3, KS_R3, 0.0, -KS_R3, -KS_R3};
};
template <> struct TwN<8> {
  static constexpr double c[8] = {1.0, KS_R2, 0.0, -KS_R2, -1.0, -KS_R2, 0.0, KS_R2};
  static constexpr double s[8] = {0.0, KS_R2, 1.0, KS_R2, 0.0, -KS_R2, -1.0, -KS_R2};
};
template <> struct TwN<16> {
  static constexpr double c[16] = {1.0, KS_C8, KS_R2, KS_S8, 0.0, -KS_S8, -KS_R2, -KS_C8,
                                   -1.0, -KS_C8, -KS_R2, -KS_S8, 0.0, KS_S8, KS_R2, KS_C8};
  static constexpr double s[16] = {0.0, KS_S8, KS_R2, KS_C8, 1.0, KS_C8, KS_R2, KS_S8,
                                   0.0, -KS_S8, -KS_R2, -KS_C8, -1.0, -KS_C8, -KS_R2, -KS_S8};
};
#undef KS_R2
#undef KS_R3
#undef KS_C8
#undef KS_S8

// Composite radix N = N1 N2 in registers (two-factor Cooley-Tukey): with
// j = j1 + N1 j2 and k = k1 + N2 k2, X[k] = sum_j1 W_N1^(j1 k2) W_N^(j1 k1)
// sum_j2 a[j1 + N1 j2] W_N2^(j2 k1): inner size-N2 transforms, constant
// twiddles, outer size-N1 transforms.  Radix 16 = 4 x 4, 8 = 4 x 2,
// 6 = 3 x 2.
template <int N1, int N2, typename T2> struct DftComp {
  __device__ static void run(T2* a) {
    using T = decltype(a[0].x);
    constexpr int N = N1 * N2;
    T2 B[N1][N2];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
#pragma unroll
      for (int j2 = 0; j2 < N2; ++j2) B[j1][j2] = a[j1 + N1 * j2];
      Dft<N2, T2>::run(B[j1]);
#pragma unroll
      for (int k1 = 1; k1 < N2; ++k1) {
        const int m = (j1 * k1) % N;
        if (j1 > 0) B[j1][k1] = cmul(B[j1][k1], cmake<T2>(T(TwN<N>::c[m]), T(-TwN<N>::s[m])));
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < N2; ++k1) {
      T2 t[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) t[j1] = B[j1][k1];
      Dft<N1, T2>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < N1; ++k2) a[k1 + N2 * k2] = t[k2];
    }
  }
};
template <typename T2> struct Dft<6, T2> : DftComp<3, 2, T2> {};
template <typename T2> struct Dft<8, T2> : DftComp<4, 2, T2> {};
template <typename T2> struct Dft<16, T2> : DftComp<4, 4, T2> {};

// LDS layout of a plane or pencil tile: one pad element after every 16, so
// that accesses with a small power-of-two element stride (the stride-R
// writes of a first Stockham stage, stride-2 pairs) fall in different banks.
// The plane passes use it; the x-pencil tiles of pass B (contiguous batches,
// conflict-free already) do not.
template <bool PAD = true> __device__ inline int lpad(int i) { return PAD ? i + (i >> 4) : i; }
__host__ __device__ inline int lpad_size(int n) { return n + (n >> 4) + 1; }

// ---------------------------------------------------------------- Stockham
// One radix-R stage over `nbatch` transforms of length n stored in LDS with
// element stride es and batch stride bs.  Ns = product of earlier radices.
// Twiddle for input q of butterfly j: exp(-2 pi i q (j mod Ns) / (Ns R)),
// read from tw[t] = exp(-2 pi i t / n) at t = q (j mod Ns) n/(Ns R) < n.
// Work item w -> (transform b, butterfly j): adjacent lanes take adjacent
// transforms when those are the contiguous direction (bs < es), so a wave's
// LDS accesses stride by bs rather than by es (a large power of two for the
// y and x transforms, which would put every lane in one bank).
template <int R, int MAXE, bool PAD, typename T2>
__device__ __forceinline__ void stockham_stage(T2* s, int nbatch, int n, int es, int bs, int Ns,
                                      const T2* __restrict__ tw) {
  constexpr int NBF = (MAXE + R - 1) / R;
  const int nbf = n / R;
  const int total = nbatch * nbf;
  const int tstep = n / (Ns * R);
  const bool bfast = bs < es;
  T2 v[NBF][R];
  int dst[NBF];
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    const int w = threadIdx.x + u * blockDim.x;
    dst[u] = -1;
    if (w < total) {
      const int b = bfast ? w % nbatch : w / nbf;
      const int j = bfast ? w / nbatch : w - b * nbf;
      const int k = j % Ns;
      const int base = b * bs;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        T2 a = s[lpad<PAD>(base + (j + q * nbf) * es)];
        if (q > 0 && k > 0) a = cmul(a, tw[q * k * tstep]);
        v[u][q] = a;
      }
      Dft<R, T2>::run(v[u]);
      dst[u] = b * bs + ((j / Ns) * Ns * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    if (dst[u] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) s[lpad<PAD>(dst[u] + q * Ns * es)] = v[u][q];
    }
  }
  __syncthreads();
}

template <int MAXE, bool PAD = true, typename T2>
__device__ __forceinline__ void fft_batch(T2* s, int nbatch, const AxisPlan& ap, int es, int bs,
                                 const T2* __restrict__ tw) {
  int Ns = 1;
  for (int st = 0; st < ap.nst; ++st) {
    const int R = ap.rad[st];
    switch (R) {
      case 2: stockham_stage<2, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 3: stockham_stage<3, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 4: stockham_stage<4, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 5: stockham_stage<5, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 7: stockham_stage<7, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 6: stockham_stage<6, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 8: stockham_stage<8, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      case 16: stockham_stage<16, MAXE, PAD>(s, nbatch, ap.n, es, bs, Ns, tw); break;
      default: break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------- fixed sizes
// The same Stockham stage with every size a compile-time constant (length N,
// NBATCH transforms, element and batch strides ES and BS, previous radix
// product NS, NT threads): the index arithmetic folds to shifts and constant
// multiplies and the work per thread is exact.  Used for cubic grids of
// 16, 48, 96 and 112 points per axis (the benchmarked cells); other grids
// take the run-time path above.
template <int R, int N, int NBATCH, int ES, int BS, int NS, int NT, bool PAD, typename T2>
__device__ __forceinline__ void stockham_stage_ct(T2* s, const T2* __restrict__ tw) {
  constexpr int NBF = N / R;
  constexpr int TOTAL = NBATCH * NBF;
  constexpr int NIT = (TOTAL + NT - 1) / NT;
  constexpr int TSTEP = N / (NS * R);
  constexpr bool BFAST = BS < ES;
  T2 v[NIT][R];
  int dst[NIT];
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    const int w = (int)threadIdx.x + u * NT;
    dst[u] = -1;
    if (TOTAL % NT == 0 || w < TOTAL) {
      const int b = BFAST ? w % NBATCH : w / NBF;
      const int j = BFAST ? w / NBATCH : w - b * NBF;
      const int k = j % NS;
      const int base = b * BS;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        T2 a = s[lpad<PAD>(base + (j + q * NBF) * ES)];
        if (q > 0 && NS > 1 && k > 0) a = cmul(a, tw[q * k * TSTEP]);
        v[u][q] = a;
      }
      Dft<R, T2>::run(v[u]);
      dst[u] = b * BS + ((j / NS) * NS * R + k) * ES;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NIT; ++u) {
    if (TOTAL % NT == 0 || dst[u] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) s[lpad<PAD>(dst[u] + q * NS * ES)] = v[u][q];
    }
  }
  __syncthreads();
}

// radix pairs of the fixed sizes: N = R1 * R2 (R2 = 1: a single stage)
template <int N> struct CtRad;
template <> struct CtRad<16> { static constexpr int R1 = 16, R2 = 1; };
template <> struct CtRad<48> { static constexpr int R1 = 16, R2 = 3; };
template <> struct CtRad<96> { static constexpr int R1 = 16, R2 = 6; };
template <> struct CtRad<112> { static constexpr int R1 = 16, R2 = 7; };

template <int N, int NBATCH, int ES, int BS, int NT, bool PAD, typename T2>
__device__ __forceinline__ void fft_ct(T2* s, const T2* __restrict__ tw) {
  constexpr int R1 = CtRad<N>::R1, R2 = CtRad<N>::R2;
  stockham_stage_ct<R1, N, NBATCH, ES, BS, 1, NT, PAD>(s, tw);
  if constexpr (R2 > 1) stockham_stage_ct<R2, N, NBATCH, ES, BS, R1, NT, PAD>(s, tw);
}

__device__ inline int wrap_m(int k, int n) { return (2 * k < n) ? k : k - n; }

// A soft-locked band of an H-apply on the W or P block (its column is exactly
// zero): the passes skip its transforms and write zeros.
__device__ inline bool band_skipped(const Fft3& f, int band) {
  return f.skip_res != nullptr && f.skip_res[band] <= f.skip_tol;
}

// ---------------------------------------------------------------- pass A
// MODE 0: load psi.  MODE 1: load r = ax - theta x and write per-plane
// partial sums of |r|^2 to partial[band*n0 + x].
// Loads per thread in flight in the global-memory loops of the passes: a
// loop that stores each loaded value before the next load keeps one load
// per thread in flight, and the passes were then bound by memory latency
// (about 16 KB in flight per CU) rather than by bandwidth.  The loads of a
// batch are unconditional, from an index clamped into range, and so are the
// stores that consume them (a guarded use draws its load into the guarded
// block, one load in flight again): an index past the end rewrites the last
// element with its own value.  Four for FP64 in 1024-thread blocks (128
// registers per thread there), or with a compile-time plane size the whole
// plane at once (nine per thread for 96^2 points: one round trip to HBM per
// plane instead of three); two loads per value (the residual form) keep four.
template <typename T, int NT, int CN = 0> constexpr int load_batch() {
  return (sizeof(T) == 8 && NT > 256) ? (CN > 0 ? (CN * CN + NT - 1) / NT : 4) : 8;
}

template <typename T, int MAXE, int MODE, int NT, int CN = 0>
__global__ void __launch_bounds__(NT)
k_pass_a(Fft3 f, const c2<T>* __restrict__ src, const c2<T>* __restrict__ src2,
         const double* __restrict__ theta, int64_t ld, c2<T>* __restrict__ dst, int64_t ldd,
         const c2<T>* __restrict__ tw1, const c2<T>* __restrict__ tw2, double* __restrict__ partial) {
  using T2 = c2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* s = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red[NT / kWave];
  const int n0 = f.ax[0].n, n1 = f.ax[1].n, n2 = f.ax[2].n;
  const int plane = CN > 0 ? CN * CN : n1 * n2;
  const int band = blockIdx.x / n0;
  const int x = blockIdx.x - band * n0;
  const int64_t off = (int64_t)x * plane;
  const T2* in = src + band * ld + off;
  constexpr int BATCH = MODE == 1 ? load_batch<T, NT>() : load_batch<T, NT, CN>();
  if (MODE == 0 && band_skipped(f, band)) {
    T2* out = dst + band * ldd + off;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) out[i] = cmake<T2>(T(0), T(0));
    return;
  }
  // twiddle tables of the two axes, staged in LDS after the plane
  T2* st1 = s + lpad_size(plane);
  T2* st2 = st1 + n1;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) st1[i] = tw1[i];
  for (int i = threadIdx.x; i < n2; i += blockDim.x) st2[i] = tw2[i];
  double acc = 0.0;
  if (MODE == 1) {
    const T2* in2 = src2 + band * ld + off;  // x
    const T th = T(theta[band]);
    for (int i0 = threadIdx.x; i0 < plane; i0 += NT * BATCH) {
      T2 a[BATCH], b[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * NT, plane - 1);
        a[u] = in[i];
        b[u] = in2[i];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = i0 + u * NT;
        const T2 r = cmake<T2>(a[u].x - th * b[u].x, a[u].y - th * b[u].y);
        const double r2 = (double)r.x * (double)r.x + (double)r.y * (double)r.y;
        acc += i < plane ? r2 : 0.0;
        s[lpad(min(i, plane - 1))] = r;
      }
    }
  } else {
    for (int i0 = threadIdx.x; i0 < plane; i0 += NT * BATCH) {
      T2 a[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) a[u] = in[min(i0 + u * NT, plane - 1)];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) s[lpad(min(i0 + u * NT, plane - 1))] = a[u];
    }
  }
  __syncthreads();
  if constexpr (CN > 0) {
    fft_ct<CN, CN, 1, CN, NT, true>(s, st2);  // z rows
    fft_ct<CN, CN, CN, 1, NT, true>(s, st1);  // y columns
  } else {
    fft_batch<MAXE>(s, n1, f.ax[2], 1, n2, st2);  // z rows
    fft_batch<MAXE>(s, n2, f.ax[1], n2, 1, st1);  // y columns
  }
  T2* out = dst + band * ldd + off;
  for (int i = threadIdx.x; i < plane; i += blockDim.x) out[i] = s[lpad(i)];
  if (MODE == 1) {
    double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- pass B
// MODE 0: multiply by T(G) = |G + k|^2/2 (k the plan's Bloch vector, zero
// at the Gamma point).  MODE 1: multiply by the TPA factor K(T(G)/E_band).
// MODE 2: no inverse; partial[block] = sum T(G)|f(G)|^2.  MODE 3: multiply
// by the periodic Poisson kernel 4 pi / |G|^2 = 2 pi / T0(G), T0 without k
// (0 at G = 0).
template <typename T, bool WITHK = true>
__device__ inline T kinetic_of(const Fft3& f, int kx, int ky, int kz) {
  const T gx = T(f.twopi_over_L[0]) * T(wrap_m(kx, f.ax[0].n)) + (WITHK ? T(f.kvec[0]) : T(0));
  const T gy = T(f.twopi_over_L[1]) * T(wrap_m(ky, f.ax[1].n)) + (WITHK ? T(f.kvec[1]) : T(0));
  const T gz = T(f.twopi_over_L[2]) * T(wrap_m(kz, f.ax[2].n)) + (WITHK ? T(f.kvec[2]) : T(0));
  return T(0.5) * (gx * gx + gy * gy + gz * gz);
}

template <typename T> __device__ inline T tpa_factor(T x) {
  const T num = T(27) + x * (T(18) + x * (T(12) + x * T(8)));
  return num / (num + T(16) * x * x * x * x);
}

template <typename T, int MAXE, int MODE, int CN = 0, int CZC = 0>
__global__ void __launch_bounds__(kThreads)
k_pass_b(Fft3 f, c2<T>* __restrict__ buf, int64_t ld, int zc, const c2<T>* __restrict__ tw0,
         const double* __restrict__ E, double* __restrict__ partial) {
  using T2 = c2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* s = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red[kThreads / kWave];
  const int n0 = f.ax[0].n, n1 = f.ax[1].n, n2 = f.ax[2].n;
  // fixed-size path: the z-chunk width is a compile-time constant
  if constexpr (CZC > 0) zc = CZC;
  const int nzc = n2 / zc;
  int bid = blockIdx.x;
  const int zt = bid % nzc; bid /= nzc;
  const int y = bid % n1;
  const int band = bid / n1;
  const int z0 = zt * zc;
  if (MODE == 0 && band_skipped(f, band)) return;  // the zero input stays zero
  T2* base = buf + band * ld + (int64_t)y * n2 + z0;
  const int64_t xs = (int64_t)n1 * n2;
  const int tile = (CN > 0 ? CN : n0) * zc;
  constexpr int BATCH = load_batch<T, kThreads>();
  T2* st0 = s + tile;  // x-axis twiddles staged in LDS after the tile
  for (int i = threadIdx.x; i < n0; i += blockDim.x) st0[i] = tw0[i];
  for (int i0 = threadIdx.x; i0 < tile; i0 += kThreads * BATCH) {
    T2 a[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = min(i0 + u * kThreads, tile - 1);
      const int x = i / zc, z = i - x * zc;
      a[u] = base[x * xs + z];
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) s[min(i0 + u * kThreads, tile - 1)] = a[u];
  }
  __syncthreads();
  if constexpr (CN > 0)
    fft_ct<CN, CZC, CZC, 1, kThreads, false>(s, st0);
  else
    fft_batch<MAXE, false>(s, zc, f.ax[0], zc, 1, st0);
  if (MODE == 2) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int kx = i / zc, z = i - kx * zc;
      const double t = (double)kinetic_of<T>(f, kx, y, z0 + z);
      const T2 sv = s[i];
      acc += t * ((double)sv.x * sv.x + (double)sv.y * sv.y);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    return;
  }
  const T einv = (MODE == 1) ? T(1.0 / E[band]) : T(0);
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    const int kx = i / zc, z = i - kx * zc;
    const T t = kinetic_of<T, MODE != 3>(f, kx, y, z0 + z);
    const T fac = (MODE == 0)   ? t
                  : (MODE == 3) ? (t > T(0) ? T(2.0 * 3.14159265358979323846) / t : T(0))
                                : tpa_factor<T>(t * einv);
    T2 v = s[i];
    s[i] = cmake<T2>(v.x * fac, -v.y * fac);  // conj for the inverse transform
  }
  __syncthreads();
  if constexpr (CN > 0)
    fft_ct<CN, CZC, CZC, 1, kThreads, false>(s, st0);
  else
    fft_batch<MAXE, false>(s, zc, f.ax[0], zc, 1, st0);
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    const int x = i / zc, z = i - x * zc;
    T2 v = s[i];
    base[x * xs + z] = cmake<T2>(v.x, -v.y);
  }
}

// ---------------------------------------------------------------- pass C
// The input plane holds conj-free spectral data in (y, z); the inverse is
// conj(FFT(conj(.))) / Ng.
// MODE 0 (H): out = Tpsi + V psi.
// MODE 1 (preconditioner): out = mask[band] * IFFT(.), mask from res > lock_tol.
template <typename T, int MAXE, int MODE, int NT, int CN = 0>
__global__ void __launch_bounds__(NT)
k_pass_c(Fft3 f, const c2<T>* __restrict__ src, int64_t lds_, c2<T>* __restrict__ dst, int64_t ldd,
         const c2<T>* __restrict__ tw1, const c2<T>* __restrict__ tw2, const T* __restrict__ V,
         const c2<T>* __restrict__ psi, int64_t ldp, const double* __restrict__ res, double lock_tol) {
  using T2 = c2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* s = reinterpret_cast<T2*>(smem_raw);
  const int n0 = f.ax[0].n, n1 = f.ax[1].n, n2 = f.ax[2].n;
  const int plane = CN > 0 ? CN * CN : n1 * n2;
  const int band = blockIdx.x / n0;
  const int x = blockIdx.x - band * n0;
  const int64_t off = (int64_t)x * plane;
  const T2* in = src + band * lds_ + off;
  constexpr int BATCH = load_batch<T, NT, CN>();
  if (MODE == 0 && band_skipped(f, band)) {
    T2* out = dst + band * ldd + off;
    for (int i = threadIdx.x; i < plane; i += blockDim.x) out[i] = cmake<T2>(T(0), T(0));
    return;
  }
  T2* st1 = s + lpad_size(plane);  // twiddle tables staged in LDS after the plane
  T2* st2 = st1 + n1;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) st1[i] = tw1[i];
  for (int i = threadIdx.x; i < n2; i += blockDim.x) st2[i] = tw2[i];
  for (int i0 = threadIdx.x; i0 < plane; i0 += NT * BATCH) {
    T2 a[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) a[u] = in[min(i0 + u * NT, plane - 1)];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) s[lpad(min(i0 + u * NT, plane - 1))] = cconj(a[u]);
  }
  __syncthreads();
  if constexpr (CN > 0) {
    fft_ct<CN, CN, CN, 1, NT, true>(s, st1);  // y columns
    fft_ct<CN, CN, 1, CN, NT, true>(s, st2);  // z rows
  } else {
    fft_batch<MAXE>(s, n2, f.ax[1], n2, 1, st1);  // y columns
    fft_batch<MAXE>(s, n1, f.ax[2], 1, n2, st2);  // z rows
  }
  const T scale = T(1.0 / ((double)n0 * (double)n1 * (double)n2));
  T2* out = dst + band * ldd + off;
  if (MODE == 0) {
    const T2* ps = psi + band * ldp + off;
    for (int i0 = threadIdx.x; i0 < plane; i0 += NT * BATCH) {
      T2 p[BATCH];
      T vr[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * NT, plane - 1);
        p[u] = ps[i];
        vr[u] = V[off + i];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * NT, plane - 1);
        const T2 t = s[lpad(i)];
        out[i] = cmake<T2>(t.x * scale + vr[u] * p[u].x, -t.y * scale + vr[u] * p[u].y);
      }
    }
  } else {
    const T m = (res[band] > lock_tol) ? scale : T(0);
    for (int i = threadIdx.x; i < plane; i += blockDim.x) {
      T2 t = s[lpad(i)];
      out[i] = cmake<T2>(t.x * m, -t.y * m);
    }
  }
}

// ---------------------------------------------------------------- split planes
// For planes that do not fit in the LDS of a CU (FP64 above 96^2 points),
// pass A becomes k_rows (z-transforms of ry consecutive y-rows of an
// x-plane, contiguous in memory) then k_cols (y-transforms of zc2
// consecutive z-columns, stride n2), and pass C becomes k_cols on conjugated
// data then k_rows with pass C's epilogue.  Tiles of at most 4096 points,
// 256 threads, no LDS padding.
// k_rows MODE 0: load psi.  MODE 1: load r = ax - theta x, partial[block] =
// sum |r|^2.  MODE 2 (H): out = conj(t)/Ng + V psi.  MODE 3: out =
// conj(t)/Ng, zero for bands with res <= lock_tol.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads)
k_rows(Fft3 f, int ry, const c2<T>* __restrict__ src, const c2<T>* __restrict__ src2,
       const double* __restrict__ theta, int64_t ld, c2<T>* __restrict__ dst, int64_t ldd,
       const c2<T>* __restrict__ tw2, const T* __restrict__ V, const c2<T>* __restrict__ psi, int64_t ldp,
       const double* __restrict__ res, double lock_tol, double* __restrict__ partial) {
  using T2 = c2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* s = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red[kThreads / kWave];
  const int n0 = f.ax[0].n, n1 = f.ax[1].n, n2 = f.ax[2].n;
  const int nrc = n1 / ry;
  int bid = blockIdx.x;
  const int rc = bid % nrc;
  bid /= nrc;
  const int x = bid % n0;
  const int band = bid / n0;
  const int tile = ry * n2;
  const int64_t off = (int64_t)x * n1 * n2 + (int64_t)rc * ry * n2;
  if ((MODE == 0 || MODE == 2) && band_skipped(f, band)) {
    T2* out = dst + band * ldd + off;
    for (int i = threadIdx.x; i < tile; i += blockDim.x) out[i] = cmake<T2>(T(0), T(0));
    return;
  }
  T2* st2 = s + tile;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) st2[i] = tw2[i];
  const T2* in = src + band * ld + off;
  constexpr int BATCH = 8;
  double acc = 0.0;
  if (MODE == 1) {
    const T2* in2 = src2 + band * ld + off;
    const T th = T(theta[band]);
    for (int i0 = threadIdx.x; i0 < tile; i0 += kThreads * BATCH) {
      T2 a[BATCH], b[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * kThreads, tile - 1);
        a[u] = in[i];
        b[u] = in2[i];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = i0 + u * kThreads;
        const T2 r = cmake<T2>(a[u].x - th * b[u].x, a[u].y - th * b[u].y);
        const double r2 = (double)r.x * (double)r.x + (double)r.y * (double)r.y;
        acc += i < tile ? r2 : 0.0;
        s[min(i, tile - 1)] = r;
      }
    }
  } else {
    for (int i0 = threadIdx.x; i0 < tile; i0 += kThreads * BATCH) {
      T2 a[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) a[u] = in[min(i0 + u * kThreads, tile - 1)];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) s[min(i0 + u * kThreads, tile - 1)] = a[u];
    }
  }
  __syncthreads();
  fft_batch<16, false>(s, ry, f.ax[2], 1, n2, st2);
  T2* out = dst + band * ldd + off;
  if (MODE <= 1) {
    for (int i = threadIdx.x; i < tile; i += blockDim.x) out[i] = s[i];
    if (MODE == 1) {
      const double t = block_sum(acc, red);
      if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
    return;
  }
  const T scale = T(1.0 / ((double)n0 * (double)n1 * (double)n2));
  if (MODE == 2) {
    const T2* ps = psi + band * ldp + off;
    for (int i0 = threadIdx.x; i0 < tile; i0 += kThreads * BATCH) {
      T2 pv[BATCH];
      T vr[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * kThreads, tile - 1);
        pv[u] = ps[i];
        vr[u] = V[off + i];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int i = min(i0 + u * kThreads, tile - 1);
        const T2 t = s[i];
        out[i] = cmake<T2>(t.x * scale + vr[u] * pv[u].x, -t.y * scale + vr[u] * pv[u].y);
      }
    }
  } else {
    const T m = (res[band] > lock_tol) ? scale : T(0);
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const T2 t = s[i];
      out[i] = cmake<T2>(t.x * m, -t.y * m);
    }
  }
}

// y-transforms of zc2 consecutive z-columns of one x-plane, in place; CONJ:
// conjugate on load (the first half of an inverse transform).
template <typename T, bool CONJ>
__global__ void __launch_bounds__(kThreads)
k_cols(Fft3 f, int zc2, c2<T>* __restrict__ buf, int64_t ld, const c2<T>* __restrict__ tw1) {
  using T2 = c2<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* s = reinterpret_cast<T2*>(smem_raw);
  const int n0 = f.ax[0].n, n1 = f.ax[1].n, n2 = f.ax[2].n;
  const int nzc = n2 / zc2;
  int bid = blockIdx.x;
  const int zt = bid % nzc;
  bid /= nzc;
  const int x = bid % n0;
  const int band = bid / n0;
  T2* base = buf + band * ld + (int64_t)x * n1 * n2 + zt * zc2;
  const int tile = n1 * zc2;
  if (band_skipped(f, band)) return;  // zeros stay zeros (forward or inverse)
  T2* st1 = s + tile;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) st1[i] = tw1[i];
  constexpr int BATCH = 8;
  for (int i0 = threadIdx.x; i0 < tile; i0 += kThreads * BATCH) {
    T2 a[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = min(i0 + u * kThreads, tile - 1);
      const int y = i / zc2, z = i - y * zc2;
      a[u] = base[(int64_t)y * n2 + z];
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) s[min(i0 + u * kThreads, tile - 1)] = CONJ ? cconj(a[u]) : a[u];
  }
  __syncthreads();
  fft_batch<16, false>(s, zc2, f.ax[1], zc2, 1, st1);
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    const int y = i / zc2, z = i - y * zc2;
    base[(int64_t)y * n2 + z] = s[i];
  }
}

// ---------------------------------------------------------------- nonlocal
// Deterministic (no atomics, fixed summation orders).

// Sum of a value over the four 16-lane rows of a wave, in every lane:
// (row0 + row1) + (row2 + row3) for rows 0 and 1, the same sum as
// (row2 + row3) + (row0 + row1) for rows 2 and 3.  The gfx950 row swaps
// move the data in registers (an xor shuffle goes through the LDS unit):
// swapping the odd rows of a copy with the even rows of another leaves the
// even-row value in one and the odd-row value in the other, for every lane
// of the row pair; the half swap does the same for lanes 0-31 and 32-63.
__device__ __forceinline__ int2 swap_rows16(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return make_int2((int)r[0], (int)r[1]);
}
__device__ __forceinline__ int2 swap_halves32(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return make_int2((int)r[0], (int)r[1]);
}
__device__ __forceinline__ double group_sum4(double v) {
  int2 lo = swap_rows16(__double2loint(v)), hi = swap_rows16(__double2hiint(v));
  v = __hiloint2double(hi.x, lo.x) + __hiloint2double(hi.y, lo.y);
  lo = swap_halves32(__double2loint(v));
  hi = swap_halves32(__double2hiint(v));
  return __hiloint2double(hi.x, lo.x) + __hiloint2double(hi.y, lo.y);
}
__device__ __forceinline__ float group_sum4(float v) {
  int2 r = swap_rows16(__float_as_int(v));
  v = __int_as_float(r.x) + __int_as_float(r.y);
  r = swap_halves32(__float_as_int(v));
  return __int_as_float(r.x) + __int_as_float(r.y);
}

// Projection with every orbital value read once.  Block (tile k, slice of
// band tiles) keeps the tile's (tile, atom) pairs in LDS: each pair lists
// the atom's support points inside the tile (tile-local point, then the np
// values of the atom's projectors there; an atom with many points in the
// tile is cut into several pairs of a bounded size, so that waves get even
// shares), loaded once for all band tiles of
// the slice (in batches of whole pairs if they do not fit).  For each band
// tile of NBS bands the orbital values of the tile's points are staged in
// LDS (z-runs of the box, coalesced), the next band tile's values loaded
// into registers meanwhile.  Each wave takes pairs in turn: lanes split into
// NBS bands x (64 / NBS) entry groups, each group sums beta_j * psi over
// every (64 / NBS)-th entry of the pair (four entries in flight, two with
// nine projectors per atom; a fixed order), the groups are combined by a
// fixed tree (row and half swaps for 16 bands, xor shuffles otherwise), and
// the pair's partial coefficients part[row + j][band]
// (j < np) are written.  The partials of a projector are summed over its
// pairs by k_nl_reduce (tiles ascending, pieces of a pair in order): the
// result does not depend on scheduling.
constexpr int kProjThreads = 1024;
template <typename T, int NBS, int MAXP, int PV>
__global__ void __launch_bounds__(kProjThreads)
k_nl_project_tile(const c2<T>* __restrict__ psi, int64_t ld, int nb, int n1, int n2, int tx, int ty, int tz,
                  int nty, int ntz, int nx, int bt_per_block, const int32_t* __restrict__ tile_pair_ptr,
                  const int32_t* __restrict__ pair_ent_ptr, const int32_t* __restrict__ pair_boff,
                  const int32_t* __restrict__ pair_row, const uint16_t* __restrict__ ent_t,
                  const T* __restrict__ ent_beta, int budget, int maxpt, c2<T>* __restrict__ part) {
  using T2 = c2<T>;
  constexpr int ROW = NBS + 1;
  constexpr int G = kWave / NBS;  // entry groups per wave
  extern __shared__ __align__(16) unsigned char proj_raw[];
  const int k = blockIdx.x;
  const int kz = k % ntz, ky = (k / ntz) % nty, kx = k / (ntz * nty);
  const int x0 = kx * tx, y0 = ky * ty, z0 = kz * tz;
  const int P = tx * ty * tz;
  const int total = P * NBS;  // <= PV * blockDim.x (checked on the host)
  T2* sp = reinterpret_cast<T2*>(proj_raw);             // P x ROW
  T* sb = reinterpret_cast<T*>(sp + (size_t)P * ROW);   // values of a batch
  int32_t* spe = reinterpret_cast<int32_t*>(sb + budget);  // 3 (maxpt + 1): entry, value offsets, rows
  int32_t* sbo = spe + maxpt + 1;
  int32_t* srow = sbo + maxpt + 1;
  uint16_t* st = reinterpret_cast<uint16_t*>(srow + maxpt + 1);  // points of a batch
  const int q0 = tile_pair_ptr[k], npair = tile_pair_ptr[k + 1] - q0;
  for (int i = threadIdx.x; i <= npair; i += blockDim.x) {
    spe[i] = pair_ent_ptr[q0 + i];
    sbo[i] = pair_boff[q0 + i];
    srow[i] = pair_row[q0 + i];
  }
  // this thread's share of a band tile: element e = threadIdx.x + u blockDim
  // -> band e / P, tile point e % P (z fastest); points outside the grid (a
  // partial last tile) and bands past nb read a clamped valid address and
  // are stored as zero
  // per element: its grid point (roff, below 2^31 points) and code = band
  // << 16 | LDS slot, or -1 for a point outside the grid or past total
  int32_t roff[PV], code[PV];
#pragma unroll
  for (int u = 0; u < PV; ++u) {
    const int e = min((int)threadIdx.x + u * (int)blockDim.x, total - 1);
    const int b = e / P, t = e - b * P;
    const int iz = t % tz, iy = (t / tz) % ty, ix = t / (tz * ty);
    const int x = x0 + ix, y = y0 + iy, z = z0 + iz;
    const bool in = (int)threadIdx.x + u * (int)blockDim.x < total && x < nx && y < n1 && z < n2;
    roff[u] = (int32_t)(((int64_t)min(x, nx - 1) * n1 + min(y, n1 - 1)) * n2 + min(z, n2 - 1));
    code[u] = in ? (b << 16) | (t * ROW + b) : -1;
  }
  const int bt0 = blockIdx.y * bt_per_block;
  const int bt1 = min(bt0 + bt_per_block, (nb + NBS - 1) / NBS);
  T2 v[PV];
  auto load_tile = [&](int bt) {
    const int b0 = bt * NBS, nbl = min(NBS, nb - b0);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int b = code[u] >> 16;  // -1 for outside points
      const T2 x = psi[(int64_t)(b0 + min(max(b, 0), nbl - 1)) * ld + roff[u]];
      v[u] = (code[u] >= 0 && b < nbl) ? x : cmake<T2>(T(0), T(0));
    }
  };
  if (bt0 < bt1) load_tile(bt0);
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int b = lane % NBS, g = lane / NBS;
  // one batch holds every pair of the tile unless their values exceed the
  // budget; then the batches are staged again for every band tile
  const bool one_batch = npair == 0 || sbo[npair] - sbo[0] <= budget;
  auto stage_batch = [&](int qa, int qb) {
    const int ea = spe[qa], ne = spe[qb] - ea;
    const int va = sbo[qa], nv = sbo[qb] - va;
    for (int i0 = threadIdx.x; i0 < nv; i0 += blockDim.x * 4) {
      T bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) bv[u] = ent_beta[va + min(i0 + u * (int)blockDim.x, nv - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * (int)blockDim.x < nv) sb[i0 + u * blockDim.x] = bv[u];
    }
    for (int i = threadIdx.x; i < ne; i += blockDim.x) st[i] = ent_t[ea + i];
  };
  __syncthreads();  // pair pointers visible
  if (one_batch && npair > 0) stage_batch(0, npair);
  for (int bt = bt0; bt < bt1; ++bt) {
    const int b0 = bt * NBS, nbl = min(NBS, nb - b0);
    // every slot of the tile is written (points outside the grid with zero)
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = (int)threadIdx.x + u * (int)blockDim.x;
      if (e < total) {
        const int b = e / P, t = e - b * P;
        sp[t * ROW + b] = v[u];
      }
    }
    __syncthreads();
    if (bt + 1 < bt1) load_tile(bt + 1);  // in flight during this band tile's sums
    int qa = 0;
    while (qa < npair) {
      int qb = npair;
      if (!one_batch) {
        // pairs qa .. qb - 1, as many whole pairs as the budget holds (one
        // pair always fits: checked on the host)
        qb = qa + 1;
        while (qb < npair && sbo[qb + 1] - sbo[qa] <= budget) ++qb;
        stage_batch(qa, qb);
        __syncthreads();
      }
      const int ea = spe[qa], va = sbo[qa];
      // a pair's bounds are the same in every lane of its wave: held in
      // scalar registers, so that the branches on them are scalar too
      for (int q = __builtin_amdgcn_readfirstlane(qa + wv); q < qb; q += nw) {
        const int e0 = __builtin_amdgcn_readfirstlane(spe[q] - ea);
        const int e1 = __builtin_amdgcn_readfirstlane(spe[q + 1] - ea);
        const int boff = __builtin_amdgcn_readfirstlane(sbo[q] - va);
        const int np = __builtin_amdgcn_readfirstlane((sbo[q + 1] - sbo[q]) / max(e1 - e0, 1));
        const T* bq = sb + boff;
        // four projectors whose values start at an even offset: read an
        // entry's values as pairs (same sums, fewer LDS reads)
        const bool vec4 = np == 4 && (boff & 1) == 0;
        // sums in the plan's precision within a tile (FP32 for the mixed
        // plans, whose H-apply is FP32 by design); tiles are summed in FP64
        T ar[MAXP], ai[MAXP];
#pragma unroll
        for (int j = 0; j < MAXP; ++j) ar[j] = ai[j] = T(0);
        // entries in flight per group (fewer with nine accumulators); the
        // loop is compiled twice, for the paired reads and the general one,
        // and the wave takes one copy (a branch on scalars)
        constexpr int UE = MAXP > 4 ? 2 : 4;
        auto entries = [&](auto paired) {
          constexpr bool V = decltype(paired)::value;
          for (int e = e0 + g; e < e1; e += UE * G) {
            int tt[UE];
            bool okk[UE];
#pragma unroll
            for (int u = 0; u < UE; ++u) {
              okk[u] = e + u * G < e1;
              tt[u] = st[min(e + u * G, e1 - 1)];
            }
            T2 w[UE];
#pragma unroll
            for (int u = 0; u < UE; ++u) w[u] = sp[tt[u] * ROW + b];
#pragma unroll
            for (int u = 0; u < UE; ++u) {
              const int el = min(e + u * G, e1 - 1) - e0;
              if constexpr (V) {
                // the entry's four values as two pair loads
                const T2* bv = reinterpret_cast<const T2*>(bq + el * 4);
                const T2 b01 = bv[0], b23 = bv[1];
                const T be[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const T bj = okk[u] ? be[j] : T(0);
                  ar[j] += bj * w[u].x;
                  ai[j] += bj * w[u].y;
                }
              } else {
                // sums of j >= np are never written, so only the lane's own
                // mask selects (a condition on the wave-uniform np becomes a
                // branch around each load); the four-projector kernel keeps
                // it in this rarely taken copy, where dropping it spills
#pragma unroll
                for (int j = 0; j < MAXP; ++j) {
                  const bool use = MAXP == 4 ? okk[u] && j < np : okk[u];
                  const T be = use ? bq[el * np + min(j, np - 1)] : T(0);
                  ar[j] += be * w[u].x;
                  ai[j] += be * w[u].y;
                }
              }
            }
          }
        };
        if constexpr (MAXP == 4) {
          if (vec4)
            entries(std::true_type{});
          else
            entries(std::false_type{});
        } else {
          entries(std::false_type{});
        }
#pragma unroll
        for (int j = 0; j < MAXP; ++j) {
          if constexpr (NBS == 16) {
            ar[j] = group_sum4(ar[j]);
            ai[j] = group_sum4(ai[j]);
          } else {
#pragma unroll
            for (int off = NBS; off < kWave; off <<= 1) {
              ar[j] += __shfl_xor(ar[j], off, kWave);
              ai[j] += __shfl_xor(ai[j], off, kWave);
            }
          }
        }
        if (g == 0 && b < nbl) {
          const int row = srow[q];
#pragma unroll
          for (int j = 0; j < MAXP; ++j)
            if (j < np) part[(int64_t)(row + j) * nb + b0 + b] = cmake<T2>(T(ar[j]), T(ai[j]));
        }
      }
      if (!one_batch) __syncthreads();
      qa = qb;
    }
    __syncthreads();  // sums done before the next band tile overwrites sp
  }
}

// Sum over the tiles of projector p (ascending) of its partial rows
// part[row][b], in FP64.
template <typename T>
__device__ inline void nl_row_sum(const c2<T>* __restrict__ part, int nb, int p, int b,
                                  const int32_t* __restrict__ proj_pair_ptr, const int32_t* __restrict__ proj_pairs,
                                  double& re, double& im) {
  using T2 = c2<T>;
  const int j0 = proj_pair_ptr[p], j1 = proj_pair_ptr[p + 1];
  re = 0.0;
  im = 0.0;
  for (int j = j0; j < j1; j += 4) {
    T2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)proj_pairs[min(j + u, j1 - 1)] * nb + b];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j + u < j1) {
        re += (double)v[u].x;
        im += (double)v[u].y;
      }
  }
}

// dc[p][b] = D_p * (row sum of projector p).  With kpairs, thread (q, b)
// takes the pair (2q, 2q + 1) of real projectors b cos(k.d), b sin(k.d):
// the coefficient of the complex projector b exp(-i k.d) is
// c = s_cos + i s_sin, and its scatter b exp(-i k.d) D c splits into
// dc[2q] = D c on the cosine part and dc[2q + 1] = -i D c on the sine part.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_nl_reduce(const c2<T>* __restrict__ part, int nb, int nproj, const int32_t* __restrict__ proj_pair_ptr,
            const int32_t* __restrict__ proj_pairs, const T* __restrict__ D, int kpairs, c2<T>* __restrict__ dc) {
  using T2 = c2<T>;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int nrow = kpairs ? nproj / 2 : nproj;
  if (i >= (int64_t)nrow * nb) return;
  const int q = (int)(i / nb), b = (int)(i - (int64_t)q * nb);
  if (!kpairs) {
    double re, im;
    nl_row_sum<T>(part, nb, q, b, proj_pair_ptr, proj_pairs, re, im);
    const double d = (double)D[q];
    dc[(int64_t)q * nb + b] = cmake<T2>(T(d * re), T(d * im));
    return;
  }
  double cr, ci, sr, si;
  nl_row_sum<T>(part, nb, 2 * q, b, proj_pair_ptr, proj_pairs, cr, ci);
  nl_row_sum<T>(part, nb, 2 * q + 1, b, proj_pair_ptr, proj_pairs, sr, si);
  const double d = (double)D[2 * q];
  const double re = d * (cr - si), im = d * (ci + sr);
  dc[(int64_t)(2 * q) * nb + b] = cmake<T2>(T(re), T(im));
  dc[(int64_t)(2 * q + 1) * nb + b] = cmake<T2>(T(im), T(-re));
}

// Nonlocal scatter: hpsi[b][r] += sum over the entries of point r of
// beta * dc[proj][b].  A block owns kScatterPts consecutive points and NBS
// bands; the dc rows of its projectors are staged in LDS (rows padded by one
// element so that lanes reading different rows fall in different banks), and
// the entries come from the ELL table (slot-major, so a wave's loads of one
// slot are contiguous; unused slots have value 0).  dc is [projector][band].
template <typename T, int NBS>
__global__ void __launch_bounds__(kScatterPts)
k_nl_scatter(c2<T>* __restrict__ hpsi, int64_t ld, int nb, int64_t Ng, const int32_t* __restrict__ ell_ptr,
             const uint16_t* __restrict__ ell_lp, const T* __restrict__ ell_beta,
             const int32_t* __restrict__ blk_ptr, const int32_t* __restrict__ blk_proj,
             const c2<T>* __restrict__ dc) {
  using T2 = c2<T>;
  constexpr int ROW = NBS + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* sdc = reinterpret_cast<T2*>(smem_raw);
  // one-dimensional grid of point blocks x band groups, ordered so that the
  // band groups of a point block run on one XCD in a row: its ELL slots and
  // staged rows are then read from HBM once per XCD, not once per group
  const int ngr = (nb + NBS - 1) / NBS;
  const int64_t g = xcd_order(blockIdx.x, gridDim.x);
  const int64_t k = g / ngr;
  const int b0 = (int)(g % ngr) * NBS;
  const int nbl = min(NBS, nb - b0);
  const int l0 = blk_ptr[k];
  const int nl = blk_ptr[k + 1] - l0;
  // Loads below are unconditional where they can be (indices clamped into
  // range, unwanted values zeroed after loading): a guarded load is issued
  // only when the one before it has returned.  A full band tile (nbl = NBS,
  // the usual case) takes the read-modify-write of hpsi without guards.
  for (int i0 = threadIdx.x; i0 < nl * NBS; i0 += blockDim.x * 4) {
    int pj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pj[u] = blk_proj[l0 + min(i0 + u * (int)blockDim.x, nl * NBS - 1) / NBS];
    T2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min(i0 + u * (int)blockDim.x, nl * NBS - 1);
      const int b = i % NBS;
      v[u] = dc[(int64_t)pj[u] * nb + b0 + min(b, nbl - 1)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min(i0 + u * (int)blockDim.x, nl * NBS - 1);
      const int l = i / NBS, b = i - l * NBS;
      sdc[l * ROW + b] = b < nbl ? v[u] : cmake<T2>(T(0), T(0));
    }
  }
  __syncthreads();
  const int64_t r = k * kScatterPts + threadIdx.x;
  if (r >= Ng) return;
  T ax[NBS], ay[NBS];
#pragma unroll
  for (int b = 0; b < NBS; ++b) ax[b] = ay[b] = T(0);
  const int w = ell_ptr[k + 1] - ell_ptr[k];
  const int64_t base = (int64_t)ell_ptr[k] * kScatterPts + threadIdx.x;
  for (int s0 = 0; s0 < w; s0 += 4) {
    int lp[4];
    T be[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = base + (int64_t)min(s0 + u, w - 1) * kScatterPts;
      lp[u] = (int)ell_lp[e];
      be[u] = ell_beta[e];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = s0 + u < w;
      lp[u] = ok ? lp[u] : 0;
      be[u] = ok ? be[u] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T2* c = sdc + lp[u] * ROW;
#pragma unroll
      for (int b = 0; b < NBS; ++b) {
        const T2 v = c[b];
        ax[b] += be[u] * v.x;
        ay[b] += be[u] * v.y;
      }
    }
  }
  if (nbl == NBS) {
    constexpr int G = NBS < 8 ? NBS : 8;  // bands per group of loads in flight
#pragma unroll
    for (int g = 0; g < NBS; g += G) {
      T2 v[G];
#pragma unroll
      for (int b = 0; b < G; ++b) v[b] = hpsi[(int64_t)(b0 + g + b) * ld + r];
#pragma unroll
      for (int b = 0; b < G; ++b)
        hpsi[(int64_t)(b0 + g + b) * ld + r] = cmake<T2>(v[b].x + ax[g + b], v[b].y + ay[g + b]);
    }
  } else {
#pragma unroll
    for (int b = 0; b < NBS; ++b) {
      if (b < nbl) {
        T2* o = hpsi + (int64_t)(b0 + b) * ld + r;
        T2 v = *o;
        v.x += ax[b];
        v.y += ay[b];
        *o = v;
      }
    }
  }
}

// ---------------------------------------------------------------- reduce
// out[b] = scale * sum_{i<cnt} partial[b*cnt + i], sequential (deterministic).
__global__ void k_row_sum(const double* __restrict__ partial, int cnt, int nb, double scale,
                          int take_sqrt, double* __restrict__ out) {
  __shared__ double red[kThreads / kWave];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) acc += partial[(int64_t)b * cnt + i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[b] = take_sqrt ? sqrt(acc * scale) : acc * scale;
}

// ---------------------------------------------------------------- launchers
template <typename T, int MAXE, int NT, int CN = 0>
static int launch_plane_a(const ks_plan& p, int mode, const c2<T>* src, const c2<T>* src2,
                          const double* theta, int64_t ld, c2<T>* dst, int64_t ldd, int nb,
                          double* partial, hipStream_t s) {
  const auto* tw1 = static_cast<const c2<T>*>(p.tw[1]);
  const auto* tw2 = static_cast<const c2<T>*>(p.tw[2]);
  dim3 grid(nb * p.fft.ax[0].n);
  TimerScope ts(KF_PASS_A, s);
  if (mode == 0)
    hipLaunchKernelGGL((k_pass_a<T, MAXE, 0, NT, CN>), grid, dim3(NT), p.lds_plane, s, p.fft, src, src2,
                       theta, ld, dst, ldd, tw1, tw2, partial);
  else
    hipLaunchKernelGGL((k_pass_a<T, MAXE, 1, NT, CN>), grid, dim3(NT), p.lds_plane, s, p.fft, src, src2,
                       theta, ld, dst, ldd, tw1, tw2, partial);
  KS_LAUNCH_CHECK("pass A");
  return 0;
}

// Fixed-size path: cubic grids of 16, 48, 96 or 112 points per axis whose
// plan chose the block shapes the compile-time kernels assume (else 0).
static int fixed_n(const ks_plan& p) {
  const int n = p.fft.ax[0].n;
  if (p.fft.ax[1].n != n || p.fft.ax[2].n != n) return 0;
  if (n == 16 && p.plane_threads == kThreads && p.maxe_plane == 4 && p.zc == 16) return 16;
  if (n == 48 && p.plane_threads == kThreads && p.maxe_plane == 16 && p.zc == 48) return 48;
  if (n == 96 && p.plane_threads == 1024 && p.maxe_plane == 12 && p.zc == 32) return 96;
  if (n == 112 && p.plane_threads == 1024 && p.maxe_plane == 16 && p.zc == 28) return 112;
  return 0;
}

template <typename T>
static int split_a(const ks_plan& p, int mode, const c2<T>* src, const c2<T>* src2, const double* theta, int64_t ld,
                   c2<T>* dst, int64_t ldd, int nb, double* partial, hipStream_t s) {
  const int n0 = p.fft.ax[0].n, n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  const auto* tw1 = static_cast<const c2<T>*>(p.tw[1]);
  const auto* tw2 = static_cast<const c2<T>*>(p.tw[2]);
  TimerScope ts(KF_PASS_A, s);
  const dim3 gr((unsigned)(nb * n0 * (n1 / p.ry)));
  if (mode == 0)
    hipLaunchKernelGGL((k_rows<T, 0>), gr, dim3(kThreads), p.lds_rows, s, p.fft, p.ry, src, src2, theta, ld, dst, ldd,
                       tw2, nullptr, nullptr, 0, nullptr, 0.0, partial);
  else
    hipLaunchKernelGGL((k_rows<T, 1>), gr, dim3(kThreads), p.lds_rows, s, p.fft, p.ry, src, src2, theta, ld, dst, ldd,
                       tw2, nullptr, nullptr, 0, nullptr, 0.0, partial);
  KS_LAUNCH_CHECK("split pass A rows");
  hipLaunchKernelGGL((k_cols<T, false>), dim3((unsigned)(nb * n0 * (n2 / p.zc2))), dim3(kThreads), p.lds_cols, s,
                     p.fft, p.zc2, dst, ldd, tw1);
  KS_LAUNCH_CHECK("split pass A columns");
  return 0;
}

template <typename T>
static int pass_a(const ks_plan& p, int mode, const c2<T>* src, const c2<T>* src2, const double* theta,
                  int64_t ld, c2<T>* dst, int64_t ldd, int nb, double* partial, hipStream_t s) {
  if (p.split) return split_a<T>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
  switch (fixed_n(p)) {
    case 16: return launch_plane_a<T, 4, kThreads, 16>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 48: return launch_plane_a<T, 16, kThreads, 48>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 96: return launch_plane_a<T, 12, 1024, 96>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 112: return launch_plane_a<T, 16, 1024, 112>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    default: break;
  }
  if (p.plane_threads == 1024) {
    if (p.maxe_plane == 12) return launch_plane_a<T, 12, 1024>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    if (p.maxe_plane == 16) return launch_plane_a<T, 16, 1024>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    return fail(KS_E_UNSUPPORTED, "plane pass shape");
  }
  switch (p.maxe_plane) {
    case 4: return launch_plane_a<T, 4, kThreads>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 16: return launch_plane_a<T, 16, kThreads>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 48: return launch_plane_a<T, 48, kThreads>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    case 64: return launch_plane_a<T, 64, kThreads>(p, mode, src, src2, theta, ld, dst, ldd, nb, partial, s);
    default: return fail(KS_E_UNSUPPORTED, "plane too large for the LDS FFT");
  }
}

template <typename T, int MAXE, int NT, int CN = 0>
static int launch_plane_c(const ks_plan& p, int mode, const c2<T>* src, int64_t lds_, c2<T>* dst,
                          int64_t ldd, int nb, const T* V, const c2<T>* psi, int64_t ldp,
                          const c2<T>* dc, const double* res, double lock_tol, hipStream_t s) {
  const auto* tw1 = static_cast<const c2<T>*>(p.tw[1]);
  const auto* tw2 = static_cast<const c2<T>*>(p.tw[2]);
  dim3 grid(nb * p.fft.ax[0].n);
  TimerScope ts(KF_PASS_C, s);
  if (mode == 0)
    hipLaunchKernelGGL((k_pass_c<T, MAXE, 0, NT, CN>), grid, dim3(NT), p.lds_plane, s, p.fft, src, lds_,
                       dst, ldd, tw1, tw2, V, psi, ldp, res, lock_tol);
  else
    hipLaunchKernelGGL((k_pass_c<T, MAXE, 1, NT, CN>), grid, dim3(NT), p.lds_plane, s, p.fft, src, lds_,
                       dst, ldd, tw1, tw2, V, psi, ldp, res, lock_tol);
  KS_LAUNCH_CHECK("pass C");
  return 0;
}

// src is scratch: the split form transforms it in place first.
template <typename T>
static int split_c(const ks_plan& p, int mode, c2<T>* src, int64_t lds_, c2<T>* dst, int64_t ldd, int nb,
                   const T* V, const c2<T>* psi, int64_t ldp, const double* res, double lock_tol, hipStream_t s) {
  const int n0 = p.fft.ax[0].n, n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  const auto* tw1 = static_cast<const c2<T>*>(p.tw[1]);
  const auto* tw2 = static_cast<const c2<T>*>(p.tw[2]);
  TimerScope ts(KF_PASS_C, s);
  hipLaunchKernelGGL((k_cols<T, true>), dim3((unsigned)(nb * n0 * (n2 / p.zc2))), dim3(kThreads), p.lds_cols, s,
                     p.fft, p.zc2, src, lds_, tw1);
  KS_LAUNCH_CHECK("split pass C columns");
  const dim3 gr((unsigned)(nb * n0 * (n1 / p.ry)));
  if (mode == 0)
    hipLaunchKernelGGL((k_rows<T, 2>), gr, dim3(kThreads), p.lds_rows, s, p.fft, p.ry, src, nullptr, nullptr, lds_,
                       dst, ldd, tw2, V, psi, ldp, res, lock_tol, nullptr);
  else
    hipLaunchKernelGGL((k_rows<T, 3>), gr, dim3(kThreads), p.lds_rows, s, p.fft, p.ry, src, nullptr, nullptr, lds_,
                       dst, ldd, tw2, V, psi, ldp, res, lock_tol, nullptr);
  KS_LAUNCH_CHECK("split pass C rows");
  return 0;
}

template <typename T>
static int pass_c(const ks_plan& p, int mode, const c2<T>* src, int64_t lds_, c2<T>* dst, int64_t ldd,
                  int nb, const T* V, const c2<T>* psi, int64_t ldp, const c2<T>* dc,
                  const double* res, double lock_tol, hipStream_t s) {
  if (p.split)
    return split_c<T>(p, mode, const_cast<c2<T>*>(src), lds_, dst, ldd, nb, V, psi, ldp, res, lock_tol, s);
  switch (fixed_n(p)) {
    case 16: return launch_plane_c<T, 4, kThreads, 16>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 48: return launch_plane_c<T, 16, kThreads, 48>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 96: return launch_plane_c<T, 12, 1024, 96>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 112: return launch_plane_c<T, 16, 1024, 112>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    default: break;
  }
  if (p.plane_threads == 1024) {
    if (p.maxe_plane == 12)
      return launch_plane_c<T, 12, 1024>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    if (p.maxe_plane == 16)
      return launch_plane_c<T, 16, 1024>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    return fail(KS_E_UNSUPPORTED, "plane pass shape");
  }
  switch (p.maxe_plane) {
    case 4: return launch_plane_c<T, 4, kThreads>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 16: return launch_plane_c<T, 16, kThreads>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 48: return launch_plane_c<T, 48, kThreads>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    case 64: return launch_plane_c<T, 64, kThreads>(p, mode, src, lds_, dst, ldd, nb, V, psi, ldp, dc, res, lock_tol, s);
    default: return fail(KS_E_UNSUPPORTED, "plane too large for the LDS FFT");
  }
}

template <typename T, int CN, int CZC>
static void launch_pencil(const ks_plan& p, int mode, dim3 grid, c2<T>* buf, int64_t ld, const c2<T>* tw0,
                          const double* E, double* partial, hipStream_t s) {
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_pass_b<T, 16, 0, CN, CZC>), grid, dim3(kThreads), p.lds_pencil, s, p.fft, buf, ld, p.zc,
                         tw0, E, partial);
      break;
    case 1:
      hipLaunchKernelGGL((k_pass_b<T, 16, 1, CN, CZC>), grid, dim3(kThreads), p.lds_pencil, s, p.fft, buf, ld, p.zc,
                         tw0, E, partial);
      break;
    case 3:
      hipLaunchKernelGGL((k_pass_b<T, 16, 3, CN, CZC>), grid, dim3(kThreads), p.lds_pencil, s, p.fft, buf, ld, p.zc,
                         tw0, E, partial);
      break;
    default:
      hipLaunchKernelGGL((k_pass_b<T, 16, 2, CN, CZC>), grid, dim3(kThreads), p.lds_pencil, s, p.fft, buf, ld, p.zc,
                         tw0, E, partial);
      break;
  }
}

template <typename T>
static int pass_b(const ks_plan& p, int mode, c2<T>* buf, int64_t ld, int nb, const double* E,
                  double* partial, hipStream_t s) {
  const auto* tw0 = static_cast<const c2<T>*>(p.tw[0]);
  const int n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  dim3 grid(nb * n1 * (n2 / p.zc));
  TimerScope ts(KF_PASS_B, s);
  if (p.maxe_pencil != 16) return fail(KS_E_UNSUPPORTED, "pencil tile size");
  switch (fixed_n(p)) {
    case 16: launch_pencil<T, 16, 16>(p, mode, grid, buf, ld, tw0, E, partial, s); break;
    case 48: launch_pencil<T, 48, 48>(p, mode, grid, buf, ld, tw0, E, partial, s); break;
    case 96: launch_pencil<T, 96, 32>(p, mode, grid, buf, ld, tw0, E, partial, s); break;
    case 112: launch_pencil<T, 112, 28>(p, mode, grid, buf, ld, tw0, E, partial, s); break;
    default: launch_pencil<T, 0, 0>(p, mode, grid, buf, ld, tw0, E, partial, s); break;
  }
  KS_LAUNCH_CHECK("pass B");
  return 0;
}

// Band-tile width of the tiled projection: 16 bands over tiles of 256 points
// in FP64 and 512 in FP32 (70 KB of LDS either way); the rest of the LDS
// holds the tile's entries.
constexpr int kProjBands = 16;

void nl_tile_shape(int prec, const int n[3], int tdim[3]) {
  const int want[3] = {prec == KS_FP64 ? 4 : 8, 8, 8};
  for (int a = 0; a < 3; ++a) tdim[a] = std::min(want[a], n[a]);
}

size_t nl_project_lds(int tile_points, size_t real_bytes, int maxpt, int budget) {
  return (size_t)tile_points * (kProjBands + 1) * 2 * real_bytes + (size_t)budget * real_bytes +
         (size_t)3 * (maxpt + 1) * 4 + (size_t)budget * 2;
}

size_t nl_dc_bytes(const ks_plan& p, int nb) {
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  return (size_t)nb * (std::max<int64_t>(p.nproj, 1) + p.nrows) * es;
}

template <typename T>
static int nl_project(const ks_plan& p, const c2<T>* psi, int64_t ld, int nb, c2<T>* dc, hipStream_t s) {
  TimerScope ts(KF_NL_PROJECT, s);
  c2<T>* part = dc + (int64_t)p.nproj * nb;
  const int P = p.tdim[0] * p.tdim[1] * p.tdim[2];
  const size_t lds = nl_project_lds(P, sizeof(T), p.maxpt, p.budget);
  // blocks: every tile, its band tiles split into slices so that there are
  // at least two blocks per compute unit
  const int ntl = p.ntile[0] * p.ntile[1] * p.ntile[2];
  const int nbt = (int)ceil_div(nb, kProjBands);
  const int slices = std::max(1, std::min(nbt, (int)ceil_div(512, ntl)));
  const int per = (int)ceil_div(nbt, slices);
  dim3 grid((unsigned)ntl, (unsigned)ceil_div(nbt, per));
  // P x 16 values per block over 1024 threads: 4 (FP64 tiles of 256) or 8
#define KS_PROJ_LAUNCH(MAXP)                                                                                       \
  hipLaunchKernelGGL((k_nl_project_tile<T, kProjBands, MAXP, sizeof(T) == 8 ? 4 : 8>), grid, dim3(kProjThreads),  \
                     lds, s, psi, ld, nb, p.fft.ax[1].n, p.fft.ax[2].n, p.tdim[0], p.tdim[1], p.tdim[2],          \
                     p.ntile[1], p.ntile[2], p.fft.ax[0].n, per, p.tile_pair_ptr, p.pair_ent_ptr, p.pair_boff,  \
                     p.pair_row, p.ent_t, static_cast<const T*>(p.ent_beta), p.budget, p.maxpt, part)
  if (p.maxp <= 1)
    KS_PROJ_LAUNCH(1);
  else if (p.maxp <= 4)
    KS_PROJ_LAUNCH(4);
  else
    KS_PROJ_LAUNCH(9);
#undef KS_PROJ_LAUNCH
  KS_LAUNCH_CHECK("nl_project_tile");
  const int64_t tot = (int64_t)(p.kpairs ? p.nproj / 2 : p.nproj) * nb;
  hipLaunchKernelGGL((k_nl_reduce<T>), dim3((unsigned)ceil_div(tot, kThreads)), dim3(kThreads), 0, s, part, nb,
                     p.nproj, p.proj_pair_ptr, p.proj_pairs, static_cast<const T*>(p.Dcoef), p.kpairs, dc);
  KS_LAUNCH_CHECK("nl_reduce");
  return 0;
}

template <typename T, int NBS>
static void launch_scatter(const ks_plan& p, c2<T>* hpsi, int64_t ldh, int nb, const c2<T>* dc, hipStream_t s) {
  const size_t lds = (size_t)p.maxl * (NBS + 1) * sizeof(c2<T>);
  dim3 grid((unsigned)((int64_t)p.nblk * ceil_div(nb, NBS)));
  hipLaunchKernelGGL((k_nl_scatter<T, NBS>), grid, dim3(kScatterPts), lds, s, hpsi, ldh, nb, p.Ng, p.ell_ptr,
                     p.ell_lp, static_cast<const T*>(p.ell_beta), p.blk_ptr, p.blk_proj, dc);
}

// The widest band group (32 bands in FP32, 16 in FP64) whose staged
// projector rows fit in 64 KB of LDS.
template <typename T>
static int nl_scatter(const ks_plan& p, c2<T>* hpsi, int64_t ldh, int nb, const c2<T>* dc, hipStream_t s) {
  TimerScope ts(KF_NL_SCATTER, s);
  const size_t row = (size_t)p.maxl * sizeof(c2<T>);
  constexpr size_t kMax = 64 * 1024;
  if (sizeof(T) == 4 && row * 33 <= kMax)
    launch_scatter<T, 32>(p, hpsi, ldh, nb, dc, s);
  else if (row * 17 <= kMax)
    launch_scatter<T, 16>(p, hpsi, ldh, nb, dc, s);
  else if (row * 9 <= kMax)
    launch_scatter<T, 8>(p, hpsi, ldh, nb, dc, s);
  else if (row * 5 <= kMax)
    launch_scatter<T, 4>(p, hpsi, ldh, nb, dc, s);
  else
    return fail(KS_E_UNSUPPORTED, "too many projectors touch one block of grid points");
  KS_LAUNCH_CHECK("nl_scatter");
  return 0;
}

template <typename T>
int apply_h(const ks_plan& p, const T* v, const c2<T>* psi, int64_t ldp, c2<T>* hpsi, int64_t ldh, int nb,
            c2<T>* tmp, c2<T>* dc, hipStream_t s, const double* skip_res, double skip_tol) {
  int rc;
  const int64_t ldt = p.Ng;
  // the FFT passes see the skip mask through a copy of the plan's transform
  // description; the NL kernels run on every band (zero columns give zero)
  ks_plan q = p;
  q.fft.skip_res = skip_res;
  q.fft.skip_tol = skip_tol;
  if (p.nproj > 0 && (rc = nl_project<T>(p, psi, ldp, nb, dc, s))) return rc;
  if ((rc = pass_a<T>(q, 0, psi, nullptr, nullptr, ldp, tmp, ldt, nb, nullptr, s))) return rc;
  if ((rc = pass_b<T>(q, 0, tmp, ldt, nb, nullptr, nullptr, s))) return rc;
  if ((rc = pass_c<T>(q, 0, tmp, ldt, hpsi, ldh, nb, v, psi, ldp, dc, nullptr, 0.0, s))) return rc;
  if (p.nproj > 0 && (rc = nl_scatter<T>(p, hpsi, ldh, nb, dc, s))) return rc;
  return 0;
}

template <typename T>
int kinetic_energy(const ks_plan& p, const c2<T>* X, int64_t ld, int nb, c2<T>* tmp, double* partial,
                   double* E, hipStream_t s) {
  int rc;
  const int64_t ldt = p.Ng;
  if ((rc = pass_a<T>(p, 0, X, nullptr, nullptr, ld, tmp, ldt, nb, nullptr, s))) return rc;
  if ((rc = pass_b<T>(p, 2, tmp, ldt, nb, nullptr, partial, s))) return rc;
  const int cnt = p.fft.ax[1].n * (p.fft.ax[2].n / p.zc);
  hipLaunchKernelGGL(k_row_sum, dim3(nb), dim3(kThreads), 0, s, partial, cnt, nb, 1.0 / (double)p.Ng, 0, E);
  KS_LAUNCH_CHECK("row_sum");
  return 0;
}

template <typename T>
int precond_apply(const ks_plan& p, int kind, const c2<T>* X, const c2<T>* AX, const double* theta,
                  int64_t ld, int nb, double lock_tol, c2<T>* W, double* res, c2<T>* tmp, double* partial,
                  double* E, hipStream_t s) {
  int rc;
  const int64_t ldt = p.Ng;
  if (kind == KS_PRECOND_TPA) {
    if ((rc = kinetic_energy<T>(p, X, ld, nb, tmp, partial, E, s))) return rc;
  }
  // residual, its norms, and the forward (y,z) transform in one pass
  if ((rc = pass_a<T>(p, 1, AX, X, theta, ld, tmp, ldt, nb, partial, s))) return rc;
  hipLaunchKernelGGL(k_row_sum, dim3(nb), dim3(kThreads), 0, s, partial, p.a_parts, nb, 1.0, 1, res);
  KS_LAUNCH_CHECK("row_sum");
  // identity preconditioner: the (y,z) forward and inverse passes cancel
  if (kind == KS_PRECOND_TPA) {
    if ((rc = pass_b<T>(p, 1, tmp, ldt, nb, E, nullptr, s))) return rc;
  }
  return pass_c<T>(p, 1, tmp, ldt, W, ld, nb, nullptr, nullptr, 0, nullptr, res, lock_tol, s);
}

// Periodic Poisson solve of one real field: out = IFFT(2 pi / T(G) FFT(in))
// on complex buffers (imaginary part of in zero), through the three passes;
// `one` is a device double holding 1 (the unmasked inverse of pass C).
template <typename T>
int poisson(const ks_plan& p, const c2<T>* in, c2<T>* tmp, c2<T>* out, const double* one, hipStream_t s) {
  int rc;
  const int64_t ld = p.Ng;
  if ((rc = pass_a<T>(p, 0, in, nullptr, nullptr, ld, tmp, ld, 1, nullptr, s))) return rc;
  if ((rc = pass_b<T>(p, 3, tmp, ld, 1, nullptr, nullptr, s))) return rc;
  return pass_c<T>(p, 1, tmp, ld, out, ld, 1, nullptr, nullptr, 0, nullptr, one, 0.0, s);
}
template int poisson<double>(const ks_plan&, const double2*, double2*, double2*, const double*, hipStream_t);
template int poisson<float>(const ks_plan&, const float2*, float2*, float2*, const double*, hipStream_t);

size_t apply_h_work_bytes(const ks_plan& p, int nb) {
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  size_t tmp = (size_t)p.Ng * nb * es;
  size_t dc = nl_dc_bytes(p, nb);
  return ((tmp + 255) / 256) * 256 + ((dc + 255) / 256) * 256;
}

size_t precond_work_bytes(const ks_plan& p, int nb) {
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  size_t tmp = (size_t)p.Ng * nb * es;
  const int n0 = p.fft.ax[0].n, n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  size_t cnt = std::max<size_t>((size_t)n0, (size_t)n1 * (n2 / p.zc));
  size_t partial = (size_t)nb * cnt * 8;
  size_t E = (size_t)nb * 8;
  return ((tmp + 255) / 256) * 256 + ((partial + 255) / 256) * 256 + ((E + 255) / 256) * 256;
}

template int apply_h<double>(const ks_plan&, const double*, const double2*, int64_t, double2*, int64_t, int,
                             double2*, double2*, hipStream_t, const double*, double);
template int apply_h<float>(const ks_plan&, const float*, const float2*, int64_t, float2*, int64_t, int,
                            float2*, float2*, hipStream_t, const double*, double);
template int kinetic_energy<double>(const ks_plan&, const double2*, int64_t, int, double2*, double*, double*,
                                    hipStream_t);
template int kinetic_energy<float>(const ks_plan&, const float2*, int64_t, int, float2*, double*, double*,
                                   hipStream_t);
template int precond_apply<double>(const ks_plan&, int, const double2*, const double2*, const double*, int64_t,
                                   int, double, double2*, double*, double2*, double*, double*, hipStream_t);
template int precond_apply<float>(const ks_plan&, int, const float2*, const float2*, const double*, int64_t,
                                  int, double, float2*, double*, float2*, double*, double*, hipStream_t);

}  // namespace ks
