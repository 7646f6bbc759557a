// Real-symmetric (Gamma-point) form of the reduction step of the generalised
// eigenproblem (Eq. 1 and the paragraph after it): S = L L^T, then
// K = L^-1 H L^-T by the explicit inverse, by two triangular solves, or by a
// blocked two-sided reduction of the xSYGST type.  With real orbitals (the
// Gamma point of a real potential) every subspace matrix is real, a product
// costs a quarter of the complex one's flops and half its bytes; the
// eigensolver figure of the paper compares the real and the complex
// solvers.  Same blocking as the complex path (32-column panels with their
// inverses in LDS), real arithmetic throughout, FP64 matrix cores for the
// products.
#include <algorithm>
#include <cfloat>

#include "gemm.hpp"

namespace ks {
namespace {

constexpr int RB = 32;            // panel width
constexpr double RCHOL_TOL = 1e-14;
constexpr int RT = 64;            // output tile edge of the product
constexpr int RKC = 16;           // K chunk staged in LDS

typedef double rd4 __attribute__((ext_vector_type(4)));

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

// ------------------------------------------------------------- the product
// C = alpha op(A) op(B) + beta C, column-major, op 'N' or 'T'.  Four waves,
// each a 32 x 32 quadrant of the 64 x 64 tile as 2 x 2 v_mfma_f64_16x16x4
// tiles (lane l holds A[l%16][l/16] and B[l/16][l%16]; result column l%16,
// rows l/16 + 4v).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_dgemm(int M, int N, int K, double alpha, const double* __restrict__ A, int lda, const double* __restrict__ B,
        int ldb, double beta, double* __restrict__ C, int ldc) {
  __shared__ double As[RKC][RT + 1];  // [k][i]
  __shared__ double Bs[RT][RKC + 1];  // [j][k]
  const int i0 = blockIdx.x * RT, j0 = blockIdx.y * RT;
  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  rd4 c[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) c[a][b][v] = 0.0;
  static_assert(RKC * RT == 4 * 256, "four elements of each tile per thread");
  for (int k0 = 0; k0 < K; k0 += RKC) {
    // four elements of each operand per thread, all eight loads issued
    // before any is used (indices clamped into range, zeroed afterwards)
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      int i, k;
      if (!TA) { i = e % RT; k = e / RT; } else { k = e % RKC; i = e / RKC; }
      const int gi = min(i0 + i, M - 1), gk = min(k0 + k, K - 1);
      av[u] = !TA ? A[gi + (int64_t)gk * lda] : A[gk + (int64_t)gi * lda];
      int j, kb;
      if (!TB) { kb = e % RKC; j = e / RKC; } else { j = e % RT; kb = e / RT; }
      const int gj = min(j0 + j, N - 1), gkb = min(k0 + kb, K - 1);
      bv[u] = !TB ? B[gkb + (int64_t)gj * ldb] : B[gj + (int64_t)gkb * ldb];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      int i, k;
      if (!TA) { i = e % RT; k = e / RT; } else { k = e % RKC; i = e / RKC; }
      As[k][i] = (i0 + i < M && k0 + k < K) ? av[u] : 0.0;
      int j, kb;
      if (!TB) { kb = e % RKC; j = e / RKC; } else { j = e % RT; kb = e / RT; }
      Bs[j][kb] = (j0 + j < N && k0 + kb < K) ? bv[u] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = As[kr][wi * 32 + u * 16 + (lane & 15)];
        b[u] = Bs[wj * 32 + u * 16 + (lane & 15)][kr];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) c[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[w], c[u][w], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wi * 32 + u * 16 + (lane >> 4) + 4 * v;
        const int gj = j0 + wj * 32 + w * 16 + (lane & 15);
        if (gi < M && gj < N) {
          double* p = C + gi + (int64_t)gj * ldc;
          *p = alpha * c[u][w][v] + (beta != 0.0 ? beta * *p : 0.0);
        }
      }
}

int dgemm(char ta, char tb, int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb,
          double beta, double* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  const dim3 grid((unsigned)ceil_div(M, RT), (unsigned)ceil_div(N, RT));
  const bool a = ta == 'T', b = tb == 'T';
  if (!a && !b)
    hipLaunchKernelGGL((k_dgemm<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (a && !b)
    hipLaunchKernelGGL((k_dgemm<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!a && b)
    hipLaunchKernelGGL((k_dgemm<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL((k_dgemm<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  KS_LAUNCH_CHECK("dgemm");
  return 0;
}

// ------------------------------------------------------------ small kernels
__global__ void k_dcopy(const double* __restrict__ src, int ld_src, double* __restrict__ dst, int ld_dst, int rows,
                        int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows);
    const int64_t j = e / rows;
    dst[i + j * ld_dst] = src[i + j * ld_src];
  }
}

unsigned grid_of(int64_t total) { return (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096); }

int dcopy(const double* src, int ld_src, double* dst, int ld_dst, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(k_dcopy, dim3(grid_of((int64_t)rows * cols)), dim3(256), 0, s, src, ld_src, dst, ld_dst, rows,
                     cols);
  KS_LAUNCH_CHECK("dcopy");
  return 0;
}

// A <- I
__global__ void k_didentity(double* __restrict__ A, int lda, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    A[i + (int64_t)j * lda] = i == j ? 1.0 : 0.0;
  }
}

// B = A^T
__global__ void k_dtranspose(const double* __restrict__ A, int lda, double* __restrict__ B, int ldb, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    B[i + (int64_t)j * ldb] = A[j + (int64_t)i * lda];
  }
}

// the strict upper triangle from the lower one
__global__ void k_dupper_from_lower(double* __restrict__ K, int ldk, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i < j) K[i + (int64_t)j * ldk] = K[j + (int64_t)i * ldk];
  }
}

// B = (A + A^T) / 2
__global__ void k_dsymmetrise_to(const double* __restrict__ A, int lda, double* __restrict__ B, int ldb, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    B[i + (int64_t)j * ldb] = 0.5 * (A[i + (int64_t)j * lda] + A[j + (int64_t)i * lda]);
  }
}

// ----------------------------------------------------------------- Cholesky
// largest diagonal entry of S (the pivot tolerance's scale); info <- 0
__global__ void k_dpotrf_init(const double* __restrict__ S, int lds, int n, double* dmax, int32_t* info) {
  __shared__ double red[4];
  double m = -DBL_MAX;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, S[i + (int64_t)i * lds]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) r = fmax(r, red[w]);
    *dmax = r;
    *info = 0;
  }
}

// Unblocked Cholesky of the kb x kb diagonal block at k0 in LDS (unscaled
// columns during the sweep, one scaling pass at the end), then the block's
// inverse, column c by lane c of the first wave.  A pivot not above
// 1e-14 max diag(S) stops the factorisation: info = info_offset + k0 + j + 1,
// and later panels return at once.
__global__ void __launch_bounds__(256)
k_dpotf2(double* __restrict__ S, int lds, int k0, int kb, const double* __restrict__ dmax, int32_t* __restrict__ info,
         int info_offset, double* __restrict__ linv) {
  __shared__ double a[RB][RB + 1];
  __shared__ double sq[RB];
  static_assert(RB * RB == 4 * 256, "four entries per thread");
  const int32_t info0 = *info;
  const double tol = RCHOL_TOL * (*dmax);
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % RB, j = e / RB;
    v[u] = S[(k0 + min(i, kb - 1)) + (int64_t)(k0 + min(j, kb - 1)) * lds];
  }
  if (info0 != 0) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % RB, j = e / RB;
    a[i][j] = (i < kb && j < kb) ? v[u] : 0.0;
  }
  __syncthreads();
  const int ri = threadIdx.x % RB, pc = threadIdx.x / RB;
  for (int j = 0; j < kb; ++j) {
    const double d = a[j][j];
    if (!(d > tol)) {
      if (threadIdx.x == 0) *info = info_offset + k0 + j + 1;
      return;  // uniform: every thread read the same pivot
    }
    const double rd = 1.0 / d;
    const double x = a[ri][j];
    double y[4], z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      y[u] = a[pc + 8 * u][j];
      z[u] = a[ri][pc + 8 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = pc + 8 * u;
      if (p > j && ri >= p && ri < kb) a[ri][p] = z[u] - x * y[u] * rd;
    }
    __syncthreads();
  }
  if (threadIdx.x < kb) sq[threadIdx.x] = sqrt(a[threadIdx.x][threadIdx.x]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % RB, j = e / RB;
    if (j < kb && i >= j && i < kb) a[i][j] = i == j ? sq[j] : a[i][j] / sq[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    const int i = e % kb, j = e / kb;
    if (i >= j) S[(k0 + i) + (int64_t)(k0 + j) * lds] = a[i][j];
  }
  if (threadIdx.x < RB) {
    const int c = threadIdx.x;
    double xc[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < i; ++p) acc += a[i][p] * xc[p];
      const bool live = c <= i && i < kb && c < kb;
      const double r = ((i == c ? 1.0 : 0.0) - acc) / a[i][i];
      xc[i] = live ? r : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) linv[i + (int64_t)c * RB] = xc[i];
  }
}

struct RealWs {
  double* dmax;
  double* linv;   // nblk x RB x RB
  double* panel;  // n x RB
  double* X;      // n x n
  double* T;      // n x n
  double* tmp;    // RB x n
  char* end;
};

RealWs real_ws(void* work, int n) {
  char* p = static_cast<char*>(work);
  RealWs w;
  w.dmax = reinterpret_cast<double*>(p);
  p += 256;
  w.linv = reinterpret_cast<double*>(p);
  p += al((size_t)ceil_div(n, RB) * RB * RB * sizeof(double));
  w.panel = reinterpret_cast<double*>(p);
  p += al((size_t)n * RB * sizeof(double));
  w.X = reinterpret_cast<double*>(p);
  p += al((size_t)n * n * sizeof(double));
  w.T = reinterpret_cast<double*>(p);
  p += al((size_t)n * n * sizeof(double));
  w.tmp = reinterpret_cast<double*>(p);
  p += al((size_t)n * RB * sizeof(double));
  w.end = p;
  return w;
}

// right-looking blocked Cholesky, lower, in place
int dpotrf(int n, double* S, int lds, const RealWs& w, int32_t* info, int info_offset, hipStream_t s) {
  hipLaunchKernelGGL(k_dpotrf_init, dim3(1), dim3(256), 0, s, S, lds, n, w.dmax, info);
  KS_LAUNCH_CHECK("dpotrf_init");
  int rc;
  for (int k0 = 0; k0 < n; k0 += RB) {
    const int kb = std::min(RB, n - k0);
    double* linv = w.linv + (size_t)(k0 / RB) * RB * RB;
    hipLaunchKernelGGL(k_dpotf2, dim3(1), dim3(256), 0, s, S, lds, k0, kb, w.dmax, info, info_offset, linv);
    KS_LAUNCH_CHECK("dpotf2");
    const int rest = n - k0 - kb;
    if (rest <= 0) break;
    double* A21 = S + (k0 + kb) + (int64_t)k0 * lds;
    // A21 <- A21 L11^-T, then A22 <- A22 - A21 A21^T
    if ((rc = dgemm('N', 'T', rest, kb, kb, 1.0, A21, lds, linv, RB, 0.0, w.panel, n, s))) return rc;
    if ((rc = dcopy(w.panel, n, A21, lds, rest, kb, s))) return rc;
    double* A22 = S + (k0 + kb) + (int64_t)(k0 + kb) * lds;
    if ((rc = dgemm('N', 'T', rest, rest, kb, -1.0, w.panel, n, w.panel, n, 1.0, A22, lds, s))) return rc;
  }
  return 0;
}

// B <- L^-1 B (L lower, n x n, from dpotrf; its inverted diagonal blocks from
// panel blk0 on), by block forward substitution
int dtrsm(int n, int ncol, const double* L, int ldl, double* B, int ldb, const RealWs& w, int blk0, hipStream_t s) {
  if (n <= 0 || ncol <= 0) return 0;
  int rc;
  const int nblk = (int)ceil_div(n, RB);
  for (int kbk = 0; kbk < nblk; ++kbk) {
    const int k0 = kbk * RB, kb = std::min(RB, n - k0);
    const double* linv = w.linv + (size_t)(blk0 + kbk) * RB * RB;
    if ((rc = dgemm('N', 'N', kb, ncol, kb, 1.0, linv, RB, B + k0, ldb, 0.0, w.tmp, RB, s))) return rc;
    if ((rc = dcopy(w.tmp, RB, B + k0, ldb, kb, ncol, s))) return rc;
    const int rest = n - k0 - kb;
    if (rest > 0)
      if ((rc = dgemm('N', 'N', rest, ncol, kb, -1.0, L + (k0 + kb) + (int64_t)k0 * ldl, ldl, w.tmp, RB, 1.0,
                      B + k0 + kb, ldb, s)))
        return rc;
  }
  return 0;
}

}  // namespace

size_t real_reduce_work(int n) {
  static char probe alignas(256);
  return (size_t)(real_ws(&probe, n).end - &probe);
}

int real_reduce_variant(int variant, int n, const double* H, int ldh, double* S, int lds_, double* K, int ldk,
                        void* work, int32_t* info, hipStream_t s) {
  const RealWs w = real_ws(work, n);
  int rc;
  if ((rc = dpotrf(n, S, lds_, w, info, n, s))) return rc;
  const double* L = S;
  const unsigned g = grid_of((int64_t)n * n);
  if (variant == 0) {
    // X = L^-1 (one solve on the identity), K = (X H) X^T
    hipLaunchKernelGGL(k_didentity, dim3(g), dim3(256), 0, s, w.X, n, n);
    if ((rc = dtrsm(n, n, L, lds_, w.X, n, w, 0, s))) return rc;
    if ((rc = dgemm('N', 'N', n, n, n, 1.0, w.X, n, H, ldh, 0.0, w.T, n, s))) return rc;
    if ((rc = dgemm('N', 'T', n, n, n, 1.0, w.T, n, w.X, n, 0.0, K, ldk, s))) return rc;
  } else if (variant == 1) {
    // Y = L^-1 H, K = L^-1 Y^T
    if ((rc = dcopy(H, ldh, w.X, n, n, n, s))) return rc;
    if ((rc = dtrsm(n, n, L, lds_, w.X, n, w, 0, s))) return rc;
    hipLaunchKernelGGL(k_dtranspose, dim3(g), dim3(256), 0, s, w.X, n, K, ldk, n);
    if ((rc = dtrsm(n, n, L, lds_, K, ldk, w, 0, s))) return rc;
  } else {
    // the blocked two-sided reduction on the lower triangle: per diagonal
    // block, A11 <- L11^-1 A11 L11^-T, A21 <- A21 L11^-T - L21 A11 / 2,
    // A22 <- A22 - A21 L21^T - L21 A21^T, A21 <- A21 - L21 A11 / 2,
    // A21 <- L22^-1 A21
    if ((rc = dcopy(H, ldh, K, ldk, n, n, s))) return rc;
    for (int k0 = 0; k0 < n; k0 += RB) {
      const int kb = std::min(RB, n - k0);
      const int r0 = k0 + kb, rest = n - r0;
      const double* linv = w.linv + (size_t)(k0 / RB) * RB * RB;
      double* A11 = K + k0 + (int64_t)k0 * ldk;
      if ((rc = dgemm('N', 'N', kb, kb, kb, 1.0, linv, RB, A11, ldk, 0.0, w.T, n, s))) return rc;
      if ((rc = dgemm('N', 'T', kb, kb, kb, 1.0, w.T, n, linv, RB, 0.0, A11, ldk, s))) return rc;
      if (rest <= 0) break;
      double* A21 = K + r0 + (int64_t)k0 * ldk;
      double* A22 = K + r0 + (int64_t)r0 * ldk;
      const double* L21 = L + r0 + (int64_t)k0 * lds_;
      const double* L22 = L + r0 + (int64_t)r0 * lds_;
      if ((rc = dgemm('N', 'T', rest, kb, kb, 1.0, A21, ldk, linv, RB, 0.0, w.X, n, s))) return rc;
      if ((rc = dgemm('N', 'N', rest, kb, kb, -0.5, L21, lds_, A11, ldk, 1.0, w.X, n, s))) return rc;
      if ((rc = dgemm('N', 'T', rest, rest, kb, -1.0, w.X, n, L21, lds_, 1.0, A22, ldk, s))) return rc;
      if ((rc = dgemm('N', 'T', rest, rest, kb, -1.0, L21, lds_, w.X, n, 1.0, A22, ldk, s))) return rc;
      if ((rc = dgemm('N', 'N', rest, kb, kb, -0.5, L21, lds_, A11, ldk, 1.0, w.X, n, s))) return rc;
      if ((rc = dtrsm(rest, kb, L22, lds_, w.X, n, w, r0 / RB, s))) return rc;
      if ((rc = dcopy(w.X, n, A21, ldk, rest, kb, s))) return rc;
    }
    hipLaunchKernelGGL(k_dupper_from_lower, dim3(g), dim3(256), 0, s, K, ldk, n);
  }
  // K <- (K + K^T) / 2, out of place through T
  hipLaunchKernelGGL(k_dsymmetrise_to, dim3(g), dim3(256), 0, s, K, ldk, w.T, n, n);
  if ((rc = dcopy(w.T, n, K, ldk, n, n, s))) return rc;
  KS_LAUNCH_CHECK("real_reduce_variant");
  return 0;
}

}  // namespace ks
