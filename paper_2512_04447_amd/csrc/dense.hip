// Dense FP64 generalised Hermitian eigensolve for the LOBPCG subspace
// problem H X = lambda S X (the paragraph before Eq. 1), by the paper's
// reduction: S = L L^H, K = L^-1 H L^-H (Eq. 1) formed with two triangular
// solves instead of a HEGST-type reduction (the paragraph after Eq. 1), a
// Hermitian eigensolve of K, and X = L^-H Z.  The triangular solves are
// products with L^-1, itself one blocked triangular solve on the identity:
// on the GPU the blocked solve is bound by its launches (three per 32-row
// block), so solving once and multiplying three times is the cheaper order.
//
// The paper calls vendor (P)ZHEEVD; here the Hermitian eigensolve is
// Householder tridiagonalisation (one column per step), bisection with
// Sturm counts for the lowest nev eigenvalues, inverse iteration with
// modified Gram-Schmidt inside clusters of close eigenvalues, and the
// back-transformation by the stored reflectors.
#include <cfloat>

#include "gemm.hpp"

namespace ks {

constexpr int NB = 32;          // panel width of the blocked factorisation
constexpr double CHOL_TOL = 1e-14;

static inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

// ---------------------------------------------------------------- potrf
__global__ void k_potrf_init(const double2* __restrict__ S, int lds, int n, double* dmax, int32_t* info,
                             int32_t* __restrict__ dead, unsigned long long* __restrict__ bound) {
  __shared__ double red[4];
  for (int i = threadIdx.x; i < n; i += blockDim.x) dead[i] = 0;
  if (threadIdx.x == 0) *bound = 0ull;
  double m = -DBL_MAX;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, S[i + (int64_t)i * lds].x);
  // block max by a fixed tree
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

// One doubling level of the inverse of the lower-triangular NB x NB
// matrix L (held in l): for each pair of S x S diagonal blocks whose
// inverses are in x, form the off-diagonal block of the inverse of the
// 2S x 2S block, -X_C (B X_A) with B the block of L below X_A and beside X_C.
// Every product runs over the whole block: the parts of X_A and X_C above
// their diagonals are zero in x.  16 S threads, one output each.
template <int S>
__device__ __forceinline__ void inverse_level(double2 (*l)[NB + 1], double2 (*x)[NB + 1], double2 (*t)[NB + 1]) {
  const int e = threadIdx.x;
  const int r0 = (e / (S * S)) * 2 * S, i = (e % (S * S)) % S, j = (e % (S * S)) / S;
  const bool act = e < 16 * S;
  if (act) {
    double accr = 0.0, acci = 0.0;
#pragma unroll
    for (int p = 0; p < S; ++p) {
      const double2 b = l[r0 + S + i][r0 + p], y = x[r0 + p][r0 + j];
      accr += b.x * y.x - b.y * y.y;
      acci += b.x * y.y + b.y * y.x;
    }
    t[r0 + S + i][r0 + j] = make_double2(accr, acci);
  }
  __syncthreads();
  if (act) {
    double accr = 0.0, acci = 0.0;
#pragma unroll
    for (int p = 0; p < S; ++p) {
      const double2 c = x[r0 + S + i][r0 + S + p], y = t[r0 + S + p][r0 + j];
      accr += c.x * y.x - c.y * y.y;
      acci += c.x * y.y + c.y * y.x;
    }
    x[r0 + S + i][r0 + j] = make_double2(-accr, -acci);
  }
  __syncthreads();
}

// Unblocked Cholesky of the diagonal block at k0 (kb <= NB columns) in LDS,
// then the inverse of that block (for the panel and the triangular solves).
// Step j updates the trailing block with the unscaled column j divided by
// the pivot d_j; no later step reads column j, so the scaling of every
// column by 1/sqrt(d_j) waits until the end (one pass, off the chain of
// steps) and a step is one LDS round trip and one barrier.
//
// A pivot not above the tolerance stops the factorisation (info) when
// dead == nullptr.  Otherwise the column is deflated: dead[k0 + j] = 1, the
// pivot becomes 1 and the column below it 0, so it takes no part in later
// columns (the live columns hold the Cholesky factor of the overlap
// restricted to them), and row j of the block's inverse is zeroed: the
// triangular solves built from these inverses then give L^-1 with zero row
// and column j, which drops basis vector j from every product with it.
__global__ void __launch_bounds__(256)
k_potf2(double2* __restrict__ S, int lds, int k0, int kb, const double* __restrict__ dmax,
        int32_t* __restrict__ info, int info_offset, double2* __restrict__ linv, int32_t* __restrict__ dead,
        int32_t* __restrict__ ndead) {
  __shared__ double2 a[NB][NB + 1];
  __shared__ double2 xa[NB][NB + 1];  // the inverse
  __shared__ double2 ta[NB][NB + 1];  // B A^-1 of the inverse's doubling
  __shared__ double sq[NB];
  __shared__ double pv[NB];  // pivots
  // the block: unconditional loads (indices clamped into the block), issued
  // together with the flag and the tolerance's scale; padding zeroed
  // afterwards, four in flight per thread
  static_assert(NB * NB == 4 * 256, "four entries per thread");
  const int32_t info0 = *info;
  const double tol = CHOL_TOL * (*dmax);
  double2 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % NB, j = e / NB;
    v[u] = S[(k0 + min(i, kb - 1)) + (int64_t)(k0 + min(j, kb - 1)) * lds];
  }
  if (info0 != 0) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % NB, j = e / NB;
    const bool in = i < kb && j < kb;
    a[i][j] = make_double2(in ? v[u].x : 0.0, in ? v[u].y : 0.0);
  }
  __syncthreads();
  // thread t owns row i = t % NB of columns p = t / NB + 8u (u = 0..3)
  const int ri = threadIdx.x % NB, pc = threadIdx.x / NB;
  const bool deflate = dead != nullptr;
  // dead columns of this block as a bit mask (the same value in every thread)
  unsigned deadmask = 0u;
  // pivot of the current step and its reciprocal, one step ahead: every
  // thread forms the next pivot from the two entries that fix it, so the
  // division runs while the step's update and barrier are in flight
  double d = a[0][0].x;
  bool dj = !(d > tol);
  double rd = dj ? 0.0 : 1.0 / d;
  for (int j = 0; j < kb; ++j) {
    if (dj && !deflate) {
      if (threadIdx.x == 0) *info = info_offset + k0 + j + 1;
      return;  // uniform: every thread holds the same pivot
    }
    deadmask |= dj ? (1u << j) : 0u;
    if (threadIdx.x == 0) pv[j] = d;
    // a[i][p] -= a[i][j] conj(a[p][j]) / d for j < p <= i < kb: every read
    // first (in range: the padding is zero), then the guarded writes; no
    // entry written here is read in this step.  A deflated column updates
    // nothing (1/d taken as 0); its entries are replaced after the loop.
    // The next pivot's entry (j+1, j+1) is read by every thread and so is
    // not written: its update is the register pivot formed below, and no
    // later step reads it from LDS.
    const int jn = min(j + 1, NB - 1);
    const double2 x = a[ri][j];
    const double dnn = a[jn][jn].x;
    const double2 xn = a[jn][j];
    double2 y[4], z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      y[u] = a[pc + 8 * u][j];
      z[u] = a[ri][pc + 8 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = pc + 8 * u;
      if (p > j && ri >= p && ri < kb && !(ri == j + 1 && p == j + 1)) {
        a[ri][p].x = z[u].x - (x.x * y[u].x + x.y * y[u].y) * rd;
        a[ri][p].y = z[u].y - (x.y * y[u].x - x.x * y[u].y) * rd;
      }
    }
    // next pivot: the same update of the entry (j+1, j+1)
    d = dnn - (xn.x * xn.x + xn.y * xn.y) * rd;
    dj = !(d > tol);
    rd = dj ? 0.0 : 1.0 / d;
    __syncthreads();
  }
  // L: column j scaled by 1/sqrt(d_j), the diagonal sqrt(d_j); a deflated
  // column becomes the unit vector (pivot 1, zeros below)
  if (dead != nullptr && threadIdx.x == 0 && deadmask != 0u) {
    for (int j = 0; j < kb; ++j)
      if ((deadmask >> j) & 1u) dead[k0 + j] = 1;
    if (ndead) atomicAdd(ndead, __popc(deadmask));
  }
  if (threadIdx.x < kb) sq[threadIdx.x] = ((deadmask >> threadIdx.x) & 1u) ? 1.0 : sqrt(pv[threadIdx.x]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % NB, j = e / NB;
    if (j < kb && i >= j && i < kb) {
      const double ljj = sq[j];
      if (i == j) {
        a[j][j] = make_double2(ljj, 0.0);
      } else if ((deadmask >> j) & 1u) {
        a[i][j] = make_double2(0.0, 0.0);
      } else {
        const double rl = 1.0 / ljj;
        a[i][j].x *= rl;
        a[i][j].y *= rl;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    const int i = e % kb, j = e / kb;
    if (i >= j) S[(k0 + i) + (int64_t)(k0 + j) * lds] = a[i][j];
  }
  // inverse X = L^-1 by doubling: with the inverses of the two diagonal
  // blocks of a lower-triangular [A 0; B C] known, the off-diagonal block of
  // its inverse is -C^-1 (B A^-1).  Block sizes 1, 2, 4, 8, 16; the padding
  // diagonal is taken as 1, and rows of dead columns or of the padding are
  // zeroed at the store (a dead column of L is a unit vector, so its column
  // of the inverse is one too and vanishes with its row).
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % NB, j = e / NB;
    const double di = i < kb ? 1.0 / sq[i] : 1.0;
    xa[i][j] = make_double2(i == j ? di : 0.0, 0.0);
  }
  __syncthreads();
  inverse_level<1>(a, xa, ta);
  inverse_level<2>(a, xa, ta);
  inverse_level<4>(a, xa, ta);
  inverse_level<8>(a, xa, ta);
  inverse_level<16>(a, xa, ta);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = e % NB, c = e / NB;
    const bool live = i < kb && ((deadmask >> i) & 1u) == 0u;
    const double2 v = xa[i][c];
    linv[e] = make_double2(live ? v.x : 0.0, live ? v.y : 0.0);
  }
}

__global__ void k_copy(const double2* __restrict__ src, int ld_src, double2* __restrict__ dst, int ld_dst, int rows,
                       int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows);
    const int64_t j = e / rows;
    dst[i + j * ld_dst] = src[i + j * ld_src];
  }
}

static int copy_block(const double2* src, int ld_src, double2* dst, int ld_dst, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return 0;
  const int64_t total = (int64_t)rows * cols;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 2048);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, src, ld_src, dst, ld_dst, rows, cols);
  KS_LAUNCH_CHECK("copy");
  return 0;
}

struct PotrfWs {
  double* dmax;
  unsigned long long* bound;  // Gershgorin bound of the reduced matrix (bits of a double >= 0)
  int32_t* dead;  // n: deflated columns
  double2* linv;  // nblk x NB x NB
  double2* panel; // n x NB
  char* end;
};

static PotrfWs potrf_ws(void* work, int n) {
  char* p = static_cast<char*>(work);
  PotrfWs w;
  w.dmax = reinterpret_cast<double*>(p);
  w.bound = reinterpret_cast<unsigned long long*>(p + 16);
  p += 256;
  w.dead = reinterpret_cast<int32_t*>(p);
  p += al((size_t)n * sizeof(int32_t));
  w.linv = reinterpret_cast<double2*>(p);
  p += al((size_t)ceil_div(n, NB) * NB * NB * sizeof(double2));
  w.panel = reinterpret_cast<double2*>(p);
  p += al((size_t)n * NB * sizeof(double2));
  w.end = p;
  return w;
}

size_t potrf_work(int n) {
  static char probe alignas(256);
  return (size_t)(potrf_ws(&probe, n).end - &probe);
}

// deflate: columns whose pivot fails are dropped (k_potf2) and counted in
// *ndead instead of stopping with info.
static int potrf_impl(int n, double2* S, int lds, void* work, int32_t* info, int info_offset, bool deflate,
                      int32_t* ndead, hipStream_t s) {
  PotrfWs w = potrf_ws(work, n);
  hipLaunchKernelGGL(k_potrf_init, dim3(1), dim3(256), 0, s, S, lds, n, w.dmax, info, w.dead, w.bound);
  KS_LAUNCH_CHECK("potrf_init");
  int rc;
  int32_t* dead = deflate ? w.dead : nullptr;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = std::min(NB, n - k0);
    double2* linv = w.linv + (size_t)(k0 / NB) * NB * NB;
    hipLaunchKernelGGL(k_potf2, dim3(1), dim3(256), 0, s, S, lds, k0, kb, w.dmax, info, info_offset, linv, dead,
                       ndead);
    KS_LAUNCH_CHECK("potf2");
    const int rest = n - k0 - kb;
    if (rest <= 0) break;
    double2* A21 = S + (k0 + kb) + (int64_t)k0 * lds;
    // panel: A21 <- A21 L_kk^-H
    if ((rc = zgemm('N', 'C', rest, kb, kb, 1.0, A21, lds, linv, NB, 0.0, w.panel, n, s))) return rc;
    if ((rc = copy_block(w.panel, n, A21, lds, rest, kb, s))) return rc;
    // trailing: A22 <- A22 - A21 A21^H (full square)
    double2* A22 = S + (k0 + kb) + (int64_t)(k0 + kb) * lds;
    if ((rc = zgemm('N', 'C', rest, rest, kb, -1.0, w.panel, n, w.panel, n, 1.0, A22, lds, s))) return rc;
  }
  return 0;
}

int potrf(int n, double2* S, int lds, void* work, int32_t* info, hipStream_t s) {
  return potrf_impl(n, S, lds, work, info, 0, false, nullptr, s);
}

int potrf_deflate(int n, double2* S, int lds, void* work, int32_t* info, int32_t* ndead, hipStream_t s) {
  return potrf_impl(n, S, lds, work, info, 0, true, ndead, s);
}

// B <- op(L)^-1 B using the inverted diagonal blocks from potrf.
// tmp: NB x ncol.
// blk0: index of L's first diagonal block among the factor's blocks (a
// trailing factor L22 starts at block blk0 of the inverted diagonal blocks).
int trsm(char op, int n, int ncol, const double2* L, int ldl, double2* B, int ldb, void* potrf_workspace, void* tmp,
         const int32_t* info, hipStream_t s, int blk0) {
  (void)info;
  if (n <= 0 || ncol <= 0) return 0;
  PotrfWs w = potrf_ws(potrf_workspace, n + blk0 * NB);
  w.linv += (size_t)blk0 * NB * NB;
  double2* T = static_cast<double2*>(tmp);
  int rc;
  const int nblk = (int)ceil_div(n, NB);
  if (op == 'N') {
    for (int kbk = 0; kbk < nblk; ++kbk) {
      const int k0 = kbk * NB, kb = std::min(NB, n - k0);
      const double2* linv = w.linv + (size_t)kbk * NB * NB;
      if ((rc = zgemm('N', 'N', kb, ncol, kb, 1.0, linv, NB, B + k0, ldb, 0.0, T, NB, s))) return rc;
      if ((rc = copy_block(T, NB, B + k0, ldb, kb, ncol, s))) return rc;
      const int rest = n - k0 - kb;
      if (rest > 0)
        if ((rc = zgemm('N', 'N', rest, ncol, kb, -1.0, L + (k0 + kb) + (int64_t)k0 * ldl, ldl, T, NB, 1.0,
                        B + k0 + kb, ldb, s)))
          return rc;
    }
  } else {
    for (int kbk = nblk - 1; kbk >= 0; --kbk) {
      const int k0 = kbk * NB, kb = std::min(NB, n - k0);
      const double2* linv = w.linv + (size_t)kbk * NB * NB;
      if ((rc = zgemm('C', 'N', kb, ncol, kb, 1.0, linv, NB, B + k0, ldb, 0.0, T, NB, s))) return rc;
      if ((rc = copy_block(T, NB, B + k0, ldb, kb, ncol, s))) return rc;
      if (k0 > 0)
        if ((rc = zgemm('C', 'N', k0, ncol, kb, -1.0, L + k0, ldl, T, NB, 1.0, B, ldb, s))) return rc;
    }
  }
  return 0;
}

// ---------------------------------------------------------------- small ops
// A <- I (n x n)
__global__ void k_set_identity(double2* __restrict__ A, int lda, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    A[i + (int64_t)j * lda] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

// K = (H + H^H)/2 out of place, one block per column j; with bound given,
// atomicMax of the column's absolute sum (the Gershgorin bound of the
// spectrum of a Hermitian K; non-negative doubles order like their bits, so
// the result does not depend on the order of the updates).
__global__ void __launch_bounds__(256)
k_hermitise_to(const double2* __restrict__ H, int ldh, double2* __restrict__ K, int ldk, int n,
               unsigned long long* __restrict__ bound) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double sum = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 a = H[i + (int64_t)j * ldh];
    const double2 b = H[j + (int64_t)i * ldh];
    const double2 m = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
    K[i + (int64_t)j * ldk] = m;
    sum += sqrt(m.x * m.x + m.y * m.y);
  }
  if (bound == nullptr) return;
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = sum;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(bound, (unsigned long long)__double_as_longlong(red[0] + red[1] + red[2] + red[3]));
}

// Deflated basis vectors: K has zero row and column j (L^-1 has), and the
// diagonal entry becomes 2 * bound + 1, above every eigenvalue of the live
// part, so the lowest eigenvectors have no component along j.
__global__ void k_deflate_diag(double2* __restrict__ K, int ldk, int n, const int32_t* __restrict__ dead,
                               const unsigned long long* __restrict__ bound) {
  const double big = 2.0 * __longlong_as_double((long long)*bound) + 1.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    if (dead[j]) K[j + (int64_t)j * ldk] = make_double2(big, 0.0);
}

// Results of the strict solve leave the workspace only when the Cholesky
// succeeded (and the tridiagonalisation's barrier did not time out).
__global__ void k_commit_results(const double* __restrict__ wsrc, double* __restrict__ w, int nev,
                                 const double2* __restrict__ Csrc, int ldcs, double2* __restrict__ C, int ldc, int n,
                                 const int32_t* __restrict__ info) {
  if (*info != 0) return;
  const int64_t total = (int64_t)n * nev;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    C[i + (int64_t)j * ldc] = Csrc[i + (int64_t)j * ldcs];
    if (i == 0) w[j] = wsrc[j];
  }
}

// ---------------------------------------------------------------- tridiagonalisation
// Step k: Householder vector of K[k+1:n, k].  With x = (alpha, x2),
// beta = -sign(Re alpha) sqrt(|alpha|^2 + |x2|^2), tau = (beta - alpha)/beta,
// v = (1, x2/(alpha - beta)), so that (I - tau v v^H)^H x = beta e_1;
// d[k] = Re K[k][k], e[k] = beta.
// Householder vector of step k fused with y = A22 v (A22 = K[k+1:, k+1:]).
// One wave per entry of y.  Every wave computes the norm of x = K[k+1:, k]
// in the same fixed order (identical results in every wave), forms
// beta, tau and v = (1, x2/(alpha - beta)) on the fly, and since A22 is
// Hermitian takes y_i = sum_j conj(A22[j][i]) v_j from the contiguous
// column i.  Wave 0 of block 0 writes v to vbuf and tau[k], d[k], e[k];
// column k of K still holds x during this kernel (the next kernel stores v
// there for the back-transform).
__global__ void __launch_bounds__(256)
k_house_hemv(const double2* __restrict__ K, int ldk, int n, int k, double2* __restrict__ tau,
             double* __restrict__ d, double* __restrict__ e, double2* __restrict__ vbuf, double2* __restrict__ y) {
  const int len = n - k - 1;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const double2* x = K + (k + 1) + (int64_t)k * ldk;
  const double2 zero = make_double2(0.0, 0.0);
  // loops take 4 loads per lane at a time so that they are in flight together
  double s = 0.0;
  for (int j0 = 1 + lane; j0 < len; j0 += 256) {
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = j0 + 64 * u < len ? x[j0 + 64 * u] : zero;
#pragma unroll
    for (int u = 0; u < 4; ++u) s += a[u].x * a[u].x + a[u].y * a[u].y;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double2 alpha = x[0];
  double2 t, scale;
  double beta;
  if (s == 0.0 && alpha.y == 0.0) {
    t = make_double2(0.0, 0.0);
    beta = alpha.x;
    scale = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + s);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double ar = alpha.x - beta, ai = alpha.y;
    const double den = ar * ar + ai * ai;
    scale = make_double2(ar / den, -ai / den);
  }
  if (row == 0) {
    for (int j = lane; j < len; j += 64) {
      const double2 xv = x[j];
      vbuf[j] = j == 0 ? make_double2(1.0, 0.0)
                       : make_double2(xv.x * scale.x - xv.y * scale.y, xv.x * scale.y + xv.y * scale.x);
    }
    if (lane == 0) {
      tau[k] = t;
      d[k] = K[k + (int64_t)k * ldk].x;
      e[k] = beta;
    }
  }
  if (row >= len) return;
  const double2* col = K + (k + 1) + (int64_t)(k + 1 + row) * ldk;
  double ar = 0.0, ai = 0.0;
  for (int j0 = lane; j0 < len; j0 += 256) {
    double2 xa[4], ca[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 64 * u;
      xa[u] = j < len ? x[j] : zero;
      ca[u] = j < len ? col[j] : zero;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + 64 * u;
      const double2 xv = xa[u];
      const double2 v = j == 0 ? make_double2(1.0, 0.0)
                               : make_double2(xv.x * scale.x - xv.y * scale.y, xv.x * scale.y + xv.y * scale.x);
      const double2 a = ca[u];
      // conj(a) v (zero beyond len)
      ar += a.x * v.x + a.y * v.y;
      ai += a.x * v.y - a.y * v.x;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  if (lane == 0) y[row] = make_double2(ar, ai);
}

// The same step for len <= 64 R with every load issued at the start: x and
// the wave's column of A22 in registers (unconditional loads from indices
// clamped into range, zeroed afterwards), so that the column does not wait
// for the norm.  Same formulas; the norm and the product are summed in
// another order.
template <int R>
__global__ void __launch_bounds__(256)
k_house_hemv_reg(const double2* __restrict__ K, int ldk, int n, int k, double2* __restrict__ tau,
                 double* __restrict__ d, double* __restrict__ e, double2* __restrict__ vbuf, double2* __restrict__ y) {
  const int len = n - k - 1;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const double2* x = K + (k + 1) + (int64_t)k * ldk;
  const double2* col = K + (k + 1) + (int64_t)(k + 1 + min(row, len - 1)) * ldk;
  double2 xa[R], ca[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int jc = min(lane + 64 * r, len - 1);
    xa[r] = x[jc];
    ca[r] = col[jc];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool in = lane + 64 * r < len;
    xa[r] = make_double2(in ? xa[r].x : 0.0, in ? xa[r].y : 0.0);
    ca[r] = make_double2(in ? ca[r].x : 0.0, in ? ca[r].y : 0.0);
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double t2 = xa[r].x * xa[r].x + xa[r].y * xa[r].y;
    s += (lane + 64 * r >= 1) ? t2 : 0.0;  // x2: entries after alpha
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double2 alpha = make_double2(__shfl(xa[0].x, 0, 64), __shfl(xa[0].y, 0, 64));
  double2 t, scale;
  double beta;
  if (s == 0.0 && alpha.y == 0.0) {
    t = make_double2(0.0, 0.0);
    beta = alpha.x;
    scale = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + s);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double ar = alpha.x - beta, ai = alpha.y;
    const double den = ar * ar + ai * ai;
    scale = make_double2(ar / den, -ai / den);
  }
  double ar = 0.0, ai = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    const double2 xv = xa[r];
    const double2 v = j == 0 ? make_double2(1.0, 0.0)
                             : make_double2(xv.x * scale.x - xv.y * scale.y, xv.x * scale.y + xv.y * scale.x);
    if (row == 0 && j < len) vbuf[j] = v;
    const double2 a = ca[r];  // zero beyond len
    ar += a.x * v.x + a.y * v.y;  // conj(a) v
    ai += a.x * v.y - a.y * v.x;
  }
  if (row == 0 && lane == 0) {
    tau[k] = t;
    d[k] = K[k + (int64_t)k * ldk].x;
    e[k] = beta;
  }
  if (row >= len) return;
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  if (lane == 0) y[row] = make_double2(ar, ai);
}

// A22 <- A22 - w v^H - v w^H with w = tau y - (1/2)|tau|^2 Re(v^H y) v.
// Every block recomputes v^H y in the same order (identical result).
// v comes from vbuf; blocks of the first column of tiles also store their
// rows of v into K[k+1:, k] (kept there for the back-transform).
__global__ void __launch_bounds__(256)
k_her2(double2* __restrict__ K, int ldk, int n, int k, const double2* __restrict__ y,
       const double2* __restrict__ tau, const double2* __restrict__ v) {
  __shared__ double red[4];
  __shared__ double2 wi_s[32], vi_s[32], wj_s[32], vj_s[32];
  const int len = n - k - 1;
  double2* A = K + (k + 1) + (int64_t)(k + 1) * ldk;
  if (blockIdx.y == 0 && threadIdx.x < 32) {
    const int i = blockIdx.x * 32 + threadIdx.x;
    if (i < len) K[(k + 1 + i) + (int64_t)k * ldk] = v[i];
  }
  const double2 t = tau[k];
  const double2 zero = make_double2(0.0, 0.0);
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  // the tile's entries do not depend on anything below: load them first.
  // Loads are unconditional from indices clamped into range, the unwanted
  // values zeroed afterwards per component (selects between addresses
  // became flat loads issued one after another).
  double2 av[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int i = i0 + (e & 31), j = j0 + (e >> 5);
    av[u] = A[min(i, len - 1) + (int64_t)min(j, len - 1) * ldk];
    const bool in = i < len && j < len;
    av[u] = make_double2(in ? av[u].x : 0.0, in ? av[u].y : 0.0);
  }
  // the 64 edge entries of v and y this block needs (rows i0.., columns j0..)
  const int qe = threadIdx.x < 32 ? i0 + threadIdx.x : j0 + (int)threadIdx.x - 32;
  const bool edge = threadIdx.x < 64 && qe < len;
  const int qc = min(qe, len - 1);
  double2 ve = v[qc], ye = y[qc];
  ve = make_double2(edge ? ve.x : 0.0, edge ? ve.y : 0.0);
  ye = make_double2(edge ? ye.x : 0.0, edge ? ye.y : 0.0);
  double s = 0.0;
  for (int q0 = threadIdx.x; q0 < len; q0 += 4 * 256) {
    double2 va[4], ya[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = min(q0 + 256 * u, len - 1);
      va[u] = v[q];
      ya[u] = y[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double t = va[u].x * ya[u].x + va[u].y * ya[u].y;  // Re(conj(v) y)
      s += q0 + 256 * u < len ? t : 0.0;
    }
  }
  s = block_sum(s, red);
  const double c = -0.5 * (t.x * t.x + t.y * t.y) * s;
  if (edge) {
    const double2 w = make_double2(t.x * ye.x - t.y * ye.y + c * ve.x, t.x * ye.y + t.y * ye.x + c * ve.y);
    if (threadIdx.x < 32) {
      vi_s[threadIdx.x] = ve;
      wi_s[threadIdx.x] = w;
    } else {
      vj_s[threadIdx.x - 32] = ve;
      wj_s[threadIdx.x - 32] = w;
    }
  }
  __syncthreads();
  // 4 entries per thread (256 threads, 32 x 32 tile), loaded at the start
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int ii = e & 31, jj = e >> 5;
    const int i = i0 + ii, j = j0 + jj;
    if (i < len && j < len) {
      const double2 wi = wi_s[ii], vi = vi_s[ii], wj = wj_s[jj], vj = vj_s[jj];
      // w_i conj(v_j) + v_i conj(w_j)
      const double re = wi.x * vj.x + wi.y * vj.y + vi.x * wj.x + vi.y * wj.y;
      const double im = wi.y * vj.x - wi.x * vj.y + vi.y * wj.x - vi.x * wj.y;
      A[i + (int64_t)j * ldk] = make_double2(av[u].x - re, av[u].y - im);
    }
  }
}

// Step k's rank-2 update (as k_her2) and step k+1's Householder vector and
// product (as k_house_hemv_reg) in one launch, for trailing sizes up to 64 R.
// Indices are those of step k's trailing matrix A22 (len x len).  One wave
// per column c = 1..len-1; column c is column c-1 of step k+1's trailing
// matrix, and the wave yields entry c-1 of y_{k+1}.  The wave loads its
// column as step k left it, v_k, y_k and column 0, forms
// w_k = tau_k y_k - (1/2)|tau_k|^2 Re(v_k^H y_k) v_k, updates column 0 and
// its own column in registers (every wave column 0 alike), takes step k+1's
// reflector from rows 1.. of the updated column 0 and its entry of y_{k+1}
// from rows 1.. of its updated column, and stores its column.  Column 0 is
// not stored: only the rows below step k+1's diagonal are used later, and
// the next launch overwrites them with v_{k+1}; d[k+1] comes from the
// registers.  Wave 0 of block 0 writes v_k into K[k+1:, k] (kept for the
// back-transform), v_{k+1}, tau[k+1], d[k+1] and e[k+1].  v and y go from
// (vin, yin) to (vout, yout), separate buffers because other waves still
// read the inputs.  No wave reads a column another wave writes.  len >= 2.
template <int R>
__global__ void __launch_bounds__(256)
k_her2_house_hemv_reg(double2* __restrict__ K, int ldk, int n, int k, double2* __restrict__ tau,
                      double* __restrict__ d, double* __restrict__ e, const double2* __restrict__ vin,
                      const double2* __restrict__ yin, double2* __restrict__ vout, double2* __restrict__ yout) {
  const int len = n - k - 1;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int c = min(row + 1, len - 1);
  double2* A = K + (k + 1) + (int64_t)(k + 1) * ldk;
  const double2 tk = tau[k];
  // every load first: unconditional, from indices clamped into range,
  // entries past len zeroed afterwards
  double2 va[R], ya[R], xa[R], ca[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int jc = min(lane + 64 * r, len - 1);
    va[r] = vin[jc];
    ya[r] = yin[jc];
    xa[r] = A[jc];
    ca[r] = A[jc + (int64_t)c * ldk];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool in = lane + 64 * r < len;
    va[r] = make_double2(in ? va[r].x : 0.0, in ? va[r].y : 0.0);
    ya[r] = make_double2(in ? ya[r].x : 0.0, in ? ya[r].y : 0.0);
    xa[r] = make_double2(in ? xa[r].x : 0.0, in ? xa[r].y : 0.0);
    ca[r] = make_double2(in ? ca[r].x : 0.0, in ? ca[r].y : 0.0);
  }
  // w_k
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) s += va[r].x * ya[r].x + va[r].y * ya[r].y;  // Re(conj(v) y)
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double cw = -0.5 * (tk.x * tk.x + tk.y * tk.y) * s;
  double2 wa[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    wa[r] = make_double2(tk.x * ya[r].x - tk.y * ya[r].y + cw * va[r].x, tk.x * ya[r].y + tk.y * ya[r].x + cw * va[r].y);
  // v and w at index 0 and at index c (register c / 64 is the same for the
  // whole wave)
  const double2 v0 = make_double2(__shfl(va[0].x, 0, 64), __shfl(va[0].y, 0, 64));
  const double2 w0 = make_double2(__shfl(wa[0].x, 0, 64), __shfl(wa[0].y, 0, 64));
  double2 vsel = va[0], wsel = wa[0];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const bool pick = (c >> 6) == r;
    vsel = make_double2(pick ? va[r].x : vsel.x, pick ? va[r].y : vsel.y);
    wsel = make_double2(pick ? wa[r].x : wsel.x, pick ? wa[r].y : wsel.y);
  }
  const double2 vc = make_double2(__shfl(vsel.x, c & 63, 64), __shfl(vsel.y, c & 63, 64));
  const double2 wc = make_double2(__shfl(wsel.x, c & 63, 64), __shfl(wsel.y, c & 63, 64));
  // A22[i][j] -= w_i conj(v_j) + v_i conj(w_j) for j = 0 and j = c
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double2 wi = wa[r], vi = va[r];
    xa[r].x -= wi.x * v0.x + wi.y * v0.y + vi.x * w0.x + vi.y * w0.y;
    xa[r].y -= wi.y * v0.x - wi.x * v0.y + vi.y * w0.x - vi.x * w0.y;
    ca[r].x -= wi.x * vc.x + wi.y * vc.y + vi.x * wc.x + vi.y * wc.y;
    ca[r].y -= wi.y * vc.x - wi.x * vc.y + vi.y * wc.x - vi.x * wc.y;
  }
  // step k+1: x = rows 1.. of column 0, alpha its first entry
  double s2 = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double t2 = xa[r].x * xa[r].x + xa[r].y * xa[r].y;
    s2 += (lane + 64 * r >= 2) ? t2 : 0.0;  // x2: entries after alpha
  }
  for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
  const double2 alpha = make_double2(__shfl(xa[0].x, 1, 64), __shfl(xa[0].y, 1, 64));
  double2 t, scale;
  double beta;
  if (s2 == 0.0 && alpha.y == 0.0) {
    t = make_double2(0.0, 0.0);
    beta = alpha.x;
    scale = make_double2(0.0, 0.0);
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + s2);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const double ar = alpha.x - beta, ai = alpha.y;
    const double den = ar * ar + ai * ai;
    scale = make_double2(ar / den, -ai / den);
  }
  const bool lead = row == 0;
  double ar = 0.0, ai = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    const double2 xv = xa[r];
    const double2 v = j == 1 ? make_double2(1.0, 0.0)
                             : make_double2(xv.x * scale.x - xv.y * scale.y, xv.x * scale.y + xv.y * scale.x);
    if (lead && j >= 1 && j < len) vout[j - 1] = v;
    if (lead && j < len) K[(k + 1 + j) + (int64_t)k * ldk] = va[r];
    const double2 a = ca[r];  // zero past len
    const bool use = j >= 1;
    ar += use ? a.x * v.x + a.y * v.y : 0.0;  // conj(a) v
    ai += use ? a.x * v.y - a.y * v.x : 0.0;
    if (row < len - 1 && j < len) A[j + (int64_t)c * ldk] = a;
  }
  if (lead && lane == 0) {
    tau[k + 1] = t;
    d[k + 1] = xa[0].x;  // updated A22[0][0]
    e[k + 1] = beta;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off, 64);
    ai += __shfl_xor(ai, off, 64);
  }
  if (row < len - 1 && lane == 0) yout[row] = make_double2(ar, ai);
}

__global__ void k_tridiag_tail(const double2* __restrict__ K, int ldk, int n, double* __restrict__ d,
                               double* __restrict__ e, double2* __restrict__ tau) {
  if (threadIdx.x == 0) {
    d[n - 1] = K[(n - 1) + (int64_t)(n - 1) * ldk].x;
    e[n - 1] = 0.0;
    tau[n - 1] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------- resident tridiagonalisation
// Steps k0..n-2 of the same reduction in one cooperative launch.  The
// trailing columns k0+1..n-1 are dealt cyclically to the G workgroups and
// stay in LDS for the whole reduction: workgroup b owns the columns
// j = k0+1 + b + q G (q < c), rows k0+1..n-1.  Step k's rank-2 update is
// not applied in step k; step k+1 applies it to each owned column just
// before that column's product with v_{k+1}, so one grid barrier per step
// suffices.  Phase k:
//  1. scalars of the pending update (step k-1): s = Re(v^H y) and
//     w = tau y - |tau|^2 s v / 2, computed by every workgroup from the same
//     data in the same order (identical in all of them);
//  2. column k of the updated matrix: its owner published it in phase k-1
//     (before the update of step k-1); the update is applied on the fly;
//  3. beta, tau_k and v_k from it, with the formulas of k_house_hemv;
//  4. every owned column j > k: pending update (rows > k), then
//     y_j = sum_i conj(A[i][j]) v_k[i]; the owner of column k+1 publishes it;
//  5. grid barrier.
// Workgroup 0 stores d, e, tau and (one phase later) v_k in column k of K,
// where the back-transform expects it.  Published vectors alternate
// between two buffers by the parity of k.
constexpr int TRI_THREADS = 256;
constexpr int TRI_RMAX = 8;  // rows per thread: trailing size <= 2048
constexpr int TRI_CMAX = 8;  // columns per workgroup
constexpr unsigned TRI_SPIN_LIMIT = 1u << 21;

// Grid barrier of a cooperative launch.  Arrivals count in two levels:
// workgroup b adds to the counter of its group b % TRI_GROUPS, and the last
// arrival of a group adds to the top counter; everyone waits for the top
// counter to reach (phase) * (number of groups).  All counters only grow
// (zeroed before the launch), so `phase` (1, 2, ...) names the wait.  The
// wait is bounded: after TRI_SPIN_LIMIT polls (well over a second) it raises
// the failure flag, and every later wait sees the flag and returns, so every
// wave reaches the end.  Layout: bar[0] top, bar[1] flag, group g's counter
// at bar[64 (g + 1)] (256 bytes apart).
constexpr int TRI_GROUPS = 8;
constexpr int TRI_BAR_WORDS = 64 * (TRI_GROUPS + 1);

__device__ bool tri_grid_barrier(unsigned* bar, unsigned phase) {
  __shared__ int ok_s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x, g = blockIdx.x % TRI_GROUPS;
    const unsigned ng = G < (unsigned)TRI_GROUPS ? G : (unsigned)TRI_GROUPS;
    const unsigned gsize = (G - g + TRI_GROUPS - 1) / TRI_GROUPS;
    int* fail = reinterpret_cast<int*>(bar + 1);
    __threadfence();
    const unsigned old =
        __hip_atomic_fetch_add(bar + 64 * (g + 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == phase * gsize) {
      __threadfence();
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    const unsigned target = phase * ng;
    for (unsigned spins = 0;; ++spins) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (spins >= TRI_SPIN_LIMIT || __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

// relaxed agent-scope load: never served by a cache that another
// workgroup's writes bypassed
__device__ inline double2 load_agent(const double2* p) {
  double* q = reinterpret_cast<double*>(const_cast<double2*>(p));
  return make_double2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a conj(b)
__device__ inline double2 zmulc2(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// bar: TRI_BAR_WORDS words, zero at launch.  On a barrier failure *info
// is set to -1.  Dynamic LDS: c m double2,
// m = n - k0 - 1.
__global__ void __launch_bounds__(TRI_THREADS)
k_tridiag_resident(double2* __restrict__ K, int ldk, int n, int k0, int c, double2* __restrict__ tau,
                   double* __restrict__ d, double* __restrict__ e, double2* __restrict__ ybuf,
                   double2* __restrict__ xbuf, unsigned* __restrict__ bar, int32_t* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char tri_raw[];
  double2* Aq = reinterpret_cast<double2*>(tri_raw);  // column q at Aq + q m
  __shared__ double red_s[TRI_THREADS / 64], red_n[TRI_THREADS / 64];
  __shared__ double2 red_y[TRI_CMAX][TRI_THREADS / 64];
  __shared__ double2 alpha_s, yk_s, xk_s, wq_s[TRI_CMAX], vq_s[TRI_CMAX];
  const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const int m = n - k0 - 1;
  const int base = k0 + 1;  // global index of local row / column 0
  const double2 zero = make_double2(0.0, 0.0);
  for (int q = 0; q < c; ++q) {
    const int jr = b + q * G;
    if (jr >= m) break;
    const double2* src = K + base + (int64_t)(base + jr) * ldk;
    // thread t owns rows t + 256 u: only it reads them back, no barrier needed
    for (int r = t; r < m; r += TRI_THREADS) Aq[q * m + r] = src[r];
  }
  double2 vp[TRI_RMAX];  // v of the pending step (zero above its head)
#pragma unroll
  for (int u = 0; u < TRI_RMAX; ++u) vp[u] = zero;
  double2 tp = zero;  // tau of the pending step
  for (int k = k0; k < n - 1; ++k) {
    const int a = k - k0;  // local index of row k+1
    const bool pend = k > k0;
    const int pin = (k - 1) & 1, pout = k & 1;
    // 1. loads: y of the pending step (rows >= k) and column k (rows > k)
    // (row k is local row a-1; its values reach the other threads through
    // LDS, written by the thread that owns the row)
    double2 y[TRI_RMAX], x[TRI_RMAX];
    if (pend) {
      const double2* yb = ybuf + (int64_t)pin * n + base;
      const double2* xb = xbuf + (int64_t)pout * n + base;
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) {
        const int r = t + TRI_THREADS * u;
        y[u] = (r >= a - 1 && r < m) ? yb[r] : zero;
        x[u] = (r >= a && r < m) ? xb[r] : zero;
        if (r == a - 1) {
          yk_s = y[u];
          xk_s = xb[r];
        }
      }
    } else {
      const double2* col = K + (int64_t)k * ldk;
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) {
        const int r = t + TRI_THREADS * u;
        y[u] = zero;
        x[u] = (r >= a && r < m) ? col[base + r] : zero;
      }
      if (t == 0) xk_s = col[k];
    }
    // 2. the pending update: w = tau y - (1/2)|tau|^2 s v, s = Re(v^H y)
    double2 w[TRI_RMAX];
    double2 wk = zero;
    if (pend) {
      double sp = 0.0;
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) sp += vp[u].x * y[u].x + vp[u].y * y[u].y;
      sp = wave_sum(sp);
      if (lane == 0) red_s[wid] = sp;
      __syncthreads();
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < TRI_THREADS / 64; ++i) s += red_s[i];
      const double c0 = -0.5 * (tp.x * tp.x + tp.y * tp.y) * s;
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) {
        const double2 ty = zmul(tp, y[u]);
        w[u] = make_double2(ty.x + c0 * vp[u].x, ty.y + c0 * vp[u].y);
      }
      // v of the pending step is exactly 1 at its head, row k
      const double2 ty = zmul(tp, yk_s);
      wk = make_double2(ty.x + c0, ty.y);
    } else {
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) w[u] = zero;
    }
    // 3. column k after the pending update: x_i - w_i - v_i conj(w_k), then
    //    the reflector of step k
    double sn = 0.0;
#pragma unroll
    for (int u = 0; u < TRI_RMAX; ++u) {
      const int r = t + TRI_THREADS * u;
      if (r >= a && r < m) {
        const double2 vw = zmulc2(vp[u], wk);
        x[u] = make_double2(x[u].x - w[u].x - vw.x, x[u].y - w[u].y - vw.y);
        if (r == a) alpha_s = x[u];
        else sn += x[u].x * x[u].x + x[u].y * x[u].y;
      }
      // the pending update's values at the rows of owned columns
      if (pend && r >= a && r < m && r >= b && (r - b) % G == 0) {
        const int q = (r - b) / G;
        wq_s[q] = w[u];
        vq_s[q] = vp[u];
      }
    }
    sn = wave_sum(sn);
    if (lane == 0) red_n[wid] = sn;
    __syncthreads();
    sn = 0.0;
#pragma unroll
    for (int i = 0; i < TRI_THREADS / 64; ++i) sn += red_n[i];
    const double2 alpha = alpha_s;
    const double dk = xk_s.x - 2.0 * wk.x;  // Re A[k][k] after the pending update
    double2 tn, scale;
    double beta;
    if (sn == 0.0 && alpha.y == 0.0) {
      tn = zero;
      beta = alpha.x;
      scale = zero;
    } else {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sn);
      beta = alpha.x >= 0.0 ? -nrm : nrm;
      tn = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      const double ar = alpha.x - beta, ai = alpha.y;
      const double den = ar * ar + ai * ai;
      scale = make_double2(ar / den, -ai / den);
    }
    double2 vn[TRI_RMAX];
#pragma unroll
    for (int u = 0; u < TRI_RMAX; ++u) {
      const int r = t + TRI_THREADS * u;
      vn[u] = r == a ? make_double2(1.0, 0.0) : (r > a && r < m) ? zmul(x[u], scale) : zero;
    }
    if (b == 0) {
      if (t == 0) {
        tau[k] = tn;
        d[k] = dk;
        e[k] = beta;
      }
      // v of the pending step into column k-1 of K (rows >= k); every
      // workgroup read that column before the previous barrier
      if (pend) {
        double2* vcol = K + base + (int64_t)(k - 1) * ldk;
#pragma unroll
        for (int u = 0; u < TRI_RMAX; ++u) {
          const int r = t + TRI_THREADS * u;
          if (r >= a - 1 && r < m) vcol[r] = vp[u];
        }
      }
    }
    // 4. owned columns j > k: pending update, then the product with v_k
    double2 acc[TRI_CMAX];
#pragma unroll
    for (int q = 0; q < TRI_CMAX; ++q) {
      acc[q] = zero;
      const int jr = b + q * G;
      if (q >= c || jr < a || jr >= m) continue;
      const double2 wj = pend ? wq_s[q] : zero, vj = pend ? vq_s[q] : zero;
      double2* col = Aq + q * m;
      double2* pub = xbuf + (int64_t)((k + 1) & 1) * n + base;
#pragma unroll
      for (int u = 0; u < TRI_RMAX; ++u) {
        const int r = t + TRI_THREADS * u;
        if (r >= a && r < m) {
          double2 A = col[r];
          if (pend) {
            const double2 p1 = zmulc2(w[u], vj), p2 = zmulc2(vp[u], wj);
            A = make_double2(A.x - p1.x - p2.x, A.y - p1.y - p2.y);
            col[r] = A;
          }
          if (jr == a) pub[r] = A;
          // conj(A) v
          acc[q].x += A.x * vn[u].x + A.y * vn[u].y;
          acc[q].y += A.x * vn[u].y - A.y * vn[u].x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < TRI_CMAX; ++q) {
      if (q >= c) break;
      const double ax = wave_sum(acc[q].x), ay = wave_sum(acc[q].y);
      if (lane == 0) red_y[q][wid] = make_double2(ax, ay);
    }
    __syncthreads();
    if (t < c) {
      const int jr = b + t * G;
      if (jr >= a && jr < m) {
        double2 sy = zero;
#pragma unroll
        for (int i = 0; i < TRI_THREADS / 64; ++i) {
          sy.x += red_y[t][i].x;
          sy.y += red_y[t][i].y;
        }
        ybuf[(int64_t)pout * n + base + jr] = sy;
      }
    }
#pragma unroll
    for (int u = 0; u < TRI_RMAX; ++u) vp[u] = vn[u];
    tp = tn;
    // 5. all of step k published
    if (!tri_grid_barrier(bar, (unsigned)(a + 1))) {
      if (t == 0) info[0] = -1;
      return;
    }
  }
  // the last diagonal entry after the update of step n-2 (v = 1 at row n-1)
  if (b == 0 && t == 0) {
    const int p = (n - 2) & 1;
    const double2 yl = load_agent(ybuf + (int64_t)p * n + (n - 1));
    const double2 xl = load_agent(xbuf + (int64_t)((n - 1) & 1) * n + (n - 1));
    const double c0 = -0.5 * (tp.x * tp.x + tp.y * tp.y) * yl.x;
    const double2 ty = zmul(tp, yl);
    d[n - 1] = xl.x - 2.0 * (ty.x + c0);
    e[n - 1] = 0.0;
    tau[n - 1] = zero;
    K[(n - 1) + (int64_t)(n - 2) * ldk] = make_double2(1.0, 0.0);
  }
}

__global__ void k_tri_reset(unsigned* bar) {
  for (int i = threadIdx.x; i < TRI_BAR_WORDS; i += blockDim.x) bar[i] = 0u;
}

// ---------------------------------------------------------------- LDS tail
// The last steps k0..n-2 of the reduction in one workgroup once the trailing
// matrix fits in LDS (m = n - k0 - 1 <= TAIL_MAX): the matrix A[k0+1:, k0+1:]
// (all of it, the step updates both triangles as k_her2 does) and column k0
// in LDS, block barriers between the parts of a step instead of two launches.
// Same formulas as k_house_hemv / k_her2 (other summation orders).  Writes
// d, e, tau for k0..n-1 and the reflectors into K's columns k0..n-2.
// Dynamic LDS: (m^2 + 4 m) double2.
constexpr int TAIL_MAX = 96;
constexpr int TAIL_THREADS = 1024;

__global__ void __launch_bounds__(TAIL_THREADS)
k_tridiag_tail_lds(double2* __restrict__ K, int ldk, int n, int k0, double2* __restrict__ tau,
                   double* __restrict__ d, double* __restrict__ e) {
  extern __shared__ __align__(16) unsigned char tail_raw[];
  const int m = n - k0 - 1;
  double2* L = reinterpret_cast<double2*>(tail_raw);  // L[i][j] = A[k0+1+i][k0+1+j], row-major
  double2* xc = L + m * m;                            // column k0, rows k0+1..
  double2* vb = xc + m;                               // reflector of the step
  double2* yb = vb + m;                               // A22 v, then w
  __shared__ double red[TAIL_THREADS / 64];
  __shared__ double2 par_s[3];                        // tau, scale, (beta, d)
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  for (int e2 = t; e2 < m * m; e2 += TAIL_THREADS) {
    const int i = e2 / m, j = e2 - i * m;
    L[e2] = K[(k0 + 1 + i) + (int64_t)(k0 + 1 + j) * ldk];
  }
  for (int i = t; i < m; i += TAIL_THREADS) xc[i] = K[(k0 + 1 + i) + (int64_t)k0 * ldk];
  const double dk0 = K[k0 + (int64_t)k0 * ldk].x;
  __syncthreads();
  for (int kk = 0; kk < m; ++kk) {
    const int k = k0 + kk, len = m - kk;
    // x = column k below the diagonal: xc for the first step, else L[kk.., kk-1]
    auto xat = [&](int i) -> double2 { return kk == 0 ? xc[i] : L[(kk + i) * m + (kk - 1)]; };
    // 1. norm of x[1:] (block reduction)
    double sp = 0.0;
    for (int i = 1 + t; i < len; i += TAIL_THREADS) {
      const double2 xv = xat(i);
      sp += xv.x * xv.x + xv.y * xv.y;
    }
    sp = wave_sum(sp);
    if (lane == 0) red[wid] = sp;
    __syncthreads();
    if (t == 0) {
      double sn = 0.0;
      for (int w = 0; w < TAIL_THREADS / 64; ++w) sn += red[w];
      const double2 alpha = xat(0);
      double2 tt, scale;
      double beta;
      if (sn == 0.0 && alpha.y == 0.0) {
        tt = make_double2(0.0, 0.0);
        beta = alpha.x;
        scale = make_double2(0.0, 0.0);
      } else {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sn);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tt = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double ar = alpha.x - beta, ai = alpha.y;
        const double den = ar * ar + ai * ai;
        scale = make_double2(ar / den, -ai / den);
      }
      par_s[0] = tt;
      par_s[1] = scale;
      tau[k] = tt;
      d[k] = kk == 0 ? dk0 : L[(kk - 1) * m + (kk - 1)].x;
      e[k] = beta;
    }
    __syncthreads();
    const double2 tt = par_s[0], scale = par_s[1];
    // 2. v = (1, x[1:] scale), into LDS and into column k of K
    for (int i = t; i < len; i += TAIL_THREADS) {
      const double2 xv = xat(i);
      const double2 v = i == 0 ? make_double2(1.0, 0.0)
                               : make_double2(xv.x * scale.x - xv.y * scale.y, xv.x * scale.y + xv.y * scale.x);
      vb[i] = v;
      K[(k + 1 + i) + (int64_t)k * ldk] = v;
    }
    __syncthreads();
    // 3. y = A22 v, y_i = sum_j conj(A22[j][i]) v_j (A22 Hermitian; column i
    //    read across consecutive threads): 8 threads per row
    {
      const int i = t >> 3, part = t & 7;
      double yr = 0.0, yi = 0.0;
      if (i < len) {
        for (int j = part; j < len; j += 8) {
          const double2 a = L[(kk + j) * m + (kk + i)];
          const double2 v = vb[j];
          yr += a.x * v.x + a.y * v.y;
          yi += a.x * v.y - a.y * v.x;
        }
      }
      for (int off = 4; off > 0; off >>= 1) {
        yr += __shfl_xor(yr, off, 8);
        yi += __shfl_xor(yi, off, 8);
      }
      if (i < len && part == 0) yb[i] = make_double2(yr, yi);
    }
    __syncthreads();
    // 4. s = Re(v^H y), w = tau y - (1/2)|tau|^2 s v
    double ss = 0.0;
    for (int i = t; i < len; i += TAIL_THREADS) ss += vb[i].x * yb[i].x + vb[i].y * yb[i].y;
    ss = wave_sum(ss);
    if (lane == 0) red[wid] = ss;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < TAIL_THREADS / 64; ++w) s += red[w];
    const double c = -0.5 * (tt.x * tt.x + tt.y * tt.y) * s;
    double2 wv = make_double2(0.0, 0.0);
    if (t < len) {
      const double2 y = yb[t], v = vb[t];
      wv = make_double2(tt.x * y.x - tt.y * y.y + c * v.x, tt.x * y.y + tt.y * y.x + c * v.y);
    }
    __syncthreads();  // every thread has read yb and red
    if (t < len) yb[t] = wv;
    __syncthreads();
    // 5. A22 <- A22 - w v^H - v w^H
    for (int e2 = t; e2 < len * len; e2 += TAIL_THREADS) {
      const int i = e2 / len, j = e2 - i * len;
      const double2 wi = yb[i], vi = vb[i], wj = yb[j], vj = vb[j];
      const double re = wi.x * vj.x + wi.y * vj.y + vi.x * wj.x + vi.y * wj.y;
      const double im = wi.y * vj.x - wi.x * vj.y + vi.y * wj.x - vi.x * wj.y;
      double2* a = L + (kk + i) * m + (kk + j);
      a->x -= re;
      a->y -= im;
    }
    __syncthreads();
  }
  if (t == 0) {
    d[n - 1] = L[(m - 1) * m + (m - 1)].x;
    e[n - 1] = 0.0;
    tau[n - 1] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------- bisection
__device__ inline double pivmin_of(const double* e, int n) {
  double m = 1.0;
  for (int i = 0; i + 1 < n; ++i) m = fmax(m, e[i] * e[i]);
  return DBL_MIN * m;
}

// Sturm count with d and e^2 staged in LDS (the recurrence carries q in a
// register; the loads do not depend on it).
__device__ inline int sturm_count_lds(const double* sd, const double* se2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = sd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = sd[i] - x - se2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Eigenvalue idx = blockIdx.x by multisection: each of the 64 lanes takes a
// Sturm count at one of 64 interior points of [lo, hi], and the interval
// shrinks to the sub-interval where the count passes idx (65x per round).
// Dynamic LDS: 2n doubles (d and e^2).
__global__ void __launch_bounds__(64)
k_bisect(const double* __restrict__ d, const double* __restrict__ e, int n, int nev, double* __restrict__ w,
         double* __restrict__ tnorm_out) {
  __shared__ int cnt[64];
  __shared__ double red[2];
  extern __shared__ __align__(16) unsigned char bis_raw[];
  double* sd = reinterpret_cast<double*>(bis_raw);
  double* se2 = sd + n;
  const int idx = blockIdx.x;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += 64) {
    sd[i] = d[i];
    se2[i] = i + 1 < n ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  double gl = DBL_MAX, gu = -DBL_MAX, em = 1.0;
  for (int i = t; i < n; i += 64) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
    if (i + 1 < n) em = fmax(em, e[i] * e[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, off, 64));
    gu = fmax(gu, __shfl_xor(gu, off, 64));
    em = fmax(em, __shfl_xor(em, off, 64));
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = DBL_MIN * em;
  double lo = gl - (2.0 * DBL_EPSILON * tnorm * n + 2.0 * pivmin);
  double hi = gu + (2.0 * DBL_EPSILON * tnorm * n + 2.0 * pivmin);
  for (int round = 0; round < 40; ++round) {
    if (hi - lo <= fmax(4.0 * DBL_EPSILON * tnorm, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) + pivmin) break;
    const double x = lo + (hi - lo) * (double)(t + 1) / 65.0;
    cnt[t] = sturm_count_lds(sd, se2, n, x, pivmin);
    __syncthreads();
    if (t == 0) {
      // first point whose count exceeds idx: the eigenvalue lies below it
      int k = 64;
      for (int q = 0; q < 64; ++q)
        if (cnt[q] > idx) { k = q; break; }
      const double nlo = k == 0 ? lo : lo + (hi - lo) * (double)k / 65.0;
      const double nhi = k == 64 ? hi : lo + (hi - lo) * (double)(k + 1) / 65.0;
      red[0] = nlo;
      red[1] = nhi;
    }
    __syncthreads();
    const double nlo = red[0], nhi = red[1];
    __syncthreads();
    if (!(nhi < hi || nlo > lo)) break;  // no progress in floating point
    lo = nlo;
    hi = nhi;
  }
  if (t == 0) {
    w[idx] = 0.5 * (lo + hi);
    if (idx == 0) *tnorm_out = tnorm;
  }
}

// Clusters of eigenvalues closer than 1e-5 ||T|| (consecutive in w): start
// indices cl[0..ncl), cl[ncl] = nev; *ncl_out = ncl.  Outside a cluster the
// inverse-iteration vectors are orthogonal to about eps ||T|| / gap <= 1e-11.
__global__ void k_clusters(const double* __restrict__ w, int nev, const double* __restrict__ tnorm,
                           int32_t* __restrict__ cl, int32_t* __restrict__ ncl_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double ortol = 1e-5 * (*tnorm);
  int ncl = 0;
  for (int i = 0; i < nev; ++i) {
    if (i == 0 || w[i] - w[i - 1] > ortol) cl[ncl++] = i;
  }
  cl[ncl] = nev;
  *ncl_out = ncl;
}

// Inverse iteration for the eigenvalues of one cluster (one block per
// cluster; blocks past the cluster count exit).  Solves (T - lambda I) x = b
// by Gaussian elimination with partial pivoting on the tridiagonal matrix
// (thread 0; the recurrences carry their running values in registers and
// store the factors in LDS), re-orthogonalises against the earlier vectors
// of the cluster whose eigenvalues lie within ortol = 1e-5 |T| of its own
// (block classical Gram-Schmidt, twice) and normalises; three sweeps.  A
// cluster is a chain of eigenvalues each within ortol of the next, and can
// span hundreds of them where the spectrum is dense; vectors of that chain
// whose eigenvalues differ by more than ortol come out orthogonal to about
// eps |T| / ortol = 1e-11 without it (the same bound the cluster test
// itself accepts between clusters), so the re-orthogonalisation is against
// the window, not the whole chain.  An ill-conditioned pencil makes |T|,
// and with it the window, large (hundreds of vectors): the dot products of
// a chunk of earlier vectors are then computed together, not one block
// reduction per vector (which cost about one second per solve for a
// window of 480).  Dynamic LDS: 5n doubles (the factor U0 (as its reciprocal), U1,
// U2, the multipliers and x) and n ints (pivots).
__global__ void __launch_bounds__(256)
k_inverse_iteration(const double* __restrict__ d, const double* __restrict__ e, int n, const double* __restrict__ w,
                    const double* __restrict__ tnorm_p, const int32_t* __restrict__ cl,
                    const int32_t* __restrict__ ncl, double* __restrict__ Z, int ldz) {
  __shared__ double red[4];
  __shared__ double lam_prev;
  __shared__ double dots[64];
  extern __shared__ __align__(16) unsigned char ii_raw[];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  double* ru0 = reinterpret_cast<double*>(ii_raw);  // 1 / U0
  double* u1 = ru0 + n;
  double* u2 = u1 + n;
  double* lm = u2 + n;
  double* x = lm + n;
  int* piv = reinterpret_cast<int*>(x + n);
  const int c = blockIdx.x;
  if (c >= *ncl) return;
  const int j0 = cl[c], j1 = cl[c + 1];
  const double tnorm = *tnorm_p;
  const double eps = DBL_EPSILON;
  const double pertol = 10.0 * eps * fmax(tnorm, DBL_MIN);
  const double small = eps * fmax(tnorm, DBL_MIN);
  const double ortol = 1e-5 * tnorm;  // the cluster test's tolerance
  for (int j = j0; j < j1; ++j) {
    double lam = w[j];
    // first earlier vector of the window: w[p] >= w[j] - ortol (w ascending;
    // the same value in every thread)
    int pbeg = j0;
    {
      int hi = j;
      const double lo_w = lam - ortol;
      while (pbeg < hi) {
        const int mid = (pbeg + hi) >> 1;
        if (w[mid] < lo_w) pbeg = mid + 1;
        else hi = mid;
      }
    }
    if (threadIdx.x == 0) {
      if (j > j0 && lam - lam_prev < pertol) lam = lam_prev + pertol;
      lam_prev = lam;
    }
    // d and e staged in LDS for the serial elimination (global loads there
    // cost a memory latency per row): d in x (written only after the
    // elimination), e in u2 (entry i is read before the elimination writes
    // it)
    double* sd = x;
    double* se = u2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      sd[i] = d[i];
      se[i] = i + 1 < n ? e[i] : 0.0;
    }
    __syncthreads();
    lam = lam_prev;
    if (threadIdx.x == 0) {
      // LU of T - lam I with partial pivoting; (c0, c1) are the diagonal and
      // superdiagonal of row i as modified by the previous elimination step
      double c0 = sd[0] - lam, c1 = n > 1 ? se[0] : 0.0;
      for (int i = 0; i + 1 < n; ++i) {
        const double b = se[i];
        const double n0 = sd[i + 1] - lam, n1 = i + 2 < n ? se[i + 1] : 0.0;
        if (fabs(c0) >= fabs(b)) {
          const double p0 = c0 == 0.0 ? small : c0;
          const double l = b / p0;
          ru0[i] = 1.0 / p0;
          u1[i] = c1;
          u2[i] = 0.0;
          lm[i] = l;
          piv[i] = 0;
          c0 = n0 - l * c1;
          c1 = n1;
        } else {
          const double l = c0 / b;
          ru0[i] = 1.0 / b;
          u1[i] = n0;
          u2[i] = n1;
          lm[i] = l;
          piv[i] = 1;
          c0 = c1 - l * n0;
          c1 = -l * n1;
        }
      }
      ru0[n - 1] = 1.0 / (c0 == 0.0 ? small : c0);
      u1[n - 1] = 0.0;
      u2[n - 1] = 0.0;
    }
    __syncthreads();  // the elimination read d from x, which is overwritten next
    // deterministic start vector
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(j * 40503u + 12345u);
      h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
      x[i] = 0.5 + (double)(h & 0xffff) / 65536.0;
    }
    __syncthreads();
    double* zj = Z + (int64_t)j * ldz;
    for (int sweep = 0; sweep < 3; ++sweep) {
      if (threadIdx.x == 0) {
        // forward: apply the row exchanges and multipliers (cur = x[i])
        double cur = x[0];
        for (int i = 0; i + 1 < n; ++i) {
          const double nx = x[i + 1], l = lm[i];
          if (piv[i] == 0) {
            x[i] = cur;
            cur = nx - l * cur;
          } else {
            x[i] = nx;
            cur = cur - l * nx;
          }
        }
        x[n - 1] = cur;
        // back substitution with U (three diagonals)
        double xa = x[n - 1] * ru0[n - 1];  // x[i+1]
        double xb = 0.0;                    // x[i+2]
        x[n - 1] = xa;
        for (int i = n - 2; i >= 0; --i) {
          const double xi = (x[i] - u1[i] * xa - u2[i] * xb) * ru0[i];
          x[i] = xi;
          xb = xa;
          xa = xi;
        }
      }
      __syncthreads();
      // scale to avoid growth, then MGS against earlier vectors of the cluster
      double mx = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(x[i]));
      for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = mx;
      __syncthreads();
      mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
      __syncthreads();
      const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] *= sc;
      __syncthreads();
      // block classical Gram-Schmidt, twice: per chunk of up to 64 earlier
      // vectors all dot products at once (wave w takes every fourth vector,
      // lanes over the rows), then one update pass over the rows
      for (int gs = 0; gs < 2; ++gs) {
        for (int c0 = pbeg; c0 < j; c0 += 64) {
          const int cn = min(64, j - c0);
          for (int q = wv; q < cn; q += 4) {
            const double* zp = Z + (int64_t)(c0 + q) * ldz;
            double dsum = 0.0;
            for (int i = ln; i < n; i += 64) dsum += zp[i] * x[i];
            dsum = wave_sum(dsum);
            if (ln == 0) dots[q] = dsum;
          }
          __syncthreads();
          for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double acc = 0.0;
            for (int q = 0; q < cn; ++q) acc += dots[q] * Z[i + (int64_t)(c0 + q) * ldz];
            x[i] -= acc;
          }
          __syncthreads();
        }
      }
      double nn = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) nn += x[i] * x[i];
      nn = block_sum(nn, red);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] *= inv;
      __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) zj[i] = x[i];
    __syncthreads();
  }
}

// C[:, j] = Q Z_T[:, j], Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^H.
// One wave per eigenvector (64-thread blocks), z in LDS: the reflector
// dot products reduce by shuffles, and the wave executes its LDS accesses in
// order, so no block barrier is needed between reflectors.
__global__ void __launch_bounds__(64)
k_backtransform(const double2* __restrict__ K, int ldk, int n, const double2* __restrict__ tau,
                const double* __restrict__ Z, int ldz, double2* __restrict__ C, int ldc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* z = reinterpret_cast<double2*>(smem_raw);
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) z[i] = make_double2(Z[i + (int64_t)j * ldz], 0.0);
  __syncthreads();
  const double2 zero = make_double2(0.0, 0.0);
  for (int k = n - 2; k >= 0; --k) {
    const double2 t = tau[k];
    if (t.x == 0.0 && t.y == 0.0) continue;  // uniform across the wave
    const double2* v = K + (k + 1) + (int64_t)k * ldk;
    double2* zk = z + k + 1;
    const int len = n - k - 1;
    double sr = 0.0, si = 0.0;
    for (int i0 = lane; i0 < len; i0 += 256) {
      double2 va[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) va[u] = i0 + 64 * u < len ? v[i0 + 64 * u] : zero;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + 64 * u < len) {
          const double2 b = zk[i0 + 64 * u];
          sr += va[u].x * b.x + va[u].y * b.y;  // conj(v) z
          si += va[u].x * b.y - va[u].y * b.x;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    // f = tau * (v^H z)
    const double fr = t.x * sr - t.y * si, fi = t.x * si + t.y * sr;
    for (int i = lane; i < len; i += 64) {
      const double2 a = v[i];
      double2 b = zk[i];
      b.x -= fr * a.x - fi * a.y;
      b.y -= fr * a.y + fi * a.x;
      zk[i] = b;
    }
    __syncthreads();  // a single wave: orders this reflector's LDS writes before the next reads
  }
  for (int i = lane; i < n; i += 64) C[i + (int64_t)j * ldc] = z[i];
}

// The same product with the reflectors in registers: lane l holds the
// entries l + 64 r (r < R) of the current reflector, uses them for both the
// dot product and the update, and loads the next reflector (k - 1) and its
// tau while the current one is applied, so that a reflector costs no
// dependent global round trip.  Global loads are unconditional from indices
// clamped into range, the reflector's entries past its length zeroed
// afterwards; the entries of z are read once per reflector, also from
// clamped indices (their products with the zeroed entries add nothing).
// Same arithmetic and summation order as k_backtransform.  n - 1 <= 64 R.
template <int R>
__global__ void __launch_bounds__(64)
k_backtransform_reg(const double2* __restrict__ K, int ldk, int n, const double2* __restrict__ tau,
                    const double* __restrict__ Z, int ldz, double2* __restrict__ C, int ldc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* z = reinterpret_cast<double2*>(smem_raw);
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) z[i] = make_double2(Z[i + (int64_t)j * ldz], 0.0);
  __syncthreads();
  double2 vc[R], vn[R];
  // reflector k: v[i'] = K[(k + 1 + i') + k ldk], i' < n - k - 1
#define KS_BT_LOAD(V, KK)                                                                      \
  do {                                                                                         \
    const int len_ = n - (KK) - 1;                                                             \
    const double2* col_ = K + ((KK) + 1) + (int64_t)(KK) * ldk;                                \
    _Pragma("unroll") for (int r = 0; r < R; ++r) V[r] = col_[min(lane + 64 * r, len_ - 1)]; \
    _Pragma("unroll") for (int r = 0; r < R; ++r) {                                            \
      const bool in_ = lane + 64 * r < len_;                                                   \
      V[r] = make_double2(in_ ? V[r].x : 0.0, in_ ? V[r].y : 0.0);                             \
    }                                                                                          \
  } while (0)
  double2 tc = make_double2(0.0, 0.0);
  if (n >= 2) {
    KS_BT_LOAD(vc, n - 2);
    tc = tau[n - 2];
  }
  for (int k = n - 2; k >= 0; --k) {
    const int kn = max(k - 1, 0);  // k = 0 reloads reflector 0 (unused)
    KS_BT_LOAD(vn, kn);
    const double2 tn = tau[kn];
    if (tc.x != 0.0 || tc.y != 0.0) {  // uniform across the wave
      const int len = n - k - 1;
      double2* zk = z + k + 1;
      // up to R = 16 the entries of z stay in registers for the update;
      // above, they are read again (registers hold two reflectors already)
      constexpr bool keep = R <= 16;
      double2 bz[keep ? R : 1];
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 b = zk[min(lane + 64 * r, len - 1)];
        if constexpr (keep) bz[r] = b;
        sr += vc[r].x * b.x + vc[r].y * b.y;  // conj(v) z
        si += vc[r].x * b.y - vc[r].y * b.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
      }
      const double fr = tc.x * sr - tc.y * si, fi = tc.x * si + tc.y * sr;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        if (i < len) {
          double2 b;
          if constexpr (keep) b = bz[r];
          else b = zk[i];
          b.x -= fr * vc[r].x - fi * vc[r].y;
          b.y -= fr * vc[r].y + fi * vc[r].x;
          zk[i] = b;
        }
      }
      __syncthreads();  // a single wave: orders this reflector's LDS writes before the next reads
    }
#pragma unroll
    for (int r = 0; r < R; ++r) vc[r] = vn[r];
    tc = tn;
  }
#undef KS_BT_LOAD
  for (int i = lane; i < n; i += 64) C[i + (int64_t)j * ldc] = z[i];
}

// ---------------------------------------------------------------- hegv
struct HegvWs {
  void* potrf;
  double2* X;  // L^-1
  double2* K;
  double2* y;
  double2* v;
  double2* tau;
  double* d;
  double* e;
  double* tnorm;
  int32_t* cl;
  int32_t* ncl;
  double* Z;
  double2* tmp;
  double2* ybuf;  // 2 n: products published by the resident tridiagonalisation
  double2* xbuf;  // 2 n: columns published by it
  unsigned* bar;  // its grid-barrier counters
  double2* y2;    // n: second y and v of the fused column steps
  double2* v2;
  double* wev;    // nev: eigenvalues before they are committed
  char* end;
};

static HegvWs hegv_ws(void* work, int n, int nev) {
  char* p = static_cast<char*>(work);
  HegvWs w;
  w.potrf = p; p += al(potrf_work(n));
  w.X = reinterpret_cast<double2*>(p); p += al((size_t)n * n * sizeof(double2));
  w.K = reinterpret_cast<double2*>(p); p += al((size_t)n * n * sizeof(double2));
  w.y = reinterpret_cast<double2*>(p); p += al((size_t)n * sizeof(double2));
  w.v = reinterpret_cast<double2*>(p); p += al((size_t)n * sizeof(double2));
  w.tau = reinterpret_cast<double2*>(p); p += al((size_t)n * sizeof(double2));
  w.d = reinterpret_cast<double*>(p); p += al((size_t)n * 8);
  w.e = reinterpret_cast<double*>(p); p += al((size_t)n * 8);
  w.tnorm = reinterpret_cast<double*>(p); p += 256;
  w.cl = reinterpret_cast<int32_t*>(p); p += al((size_t)(nev + 1) * 4);
  w.ncl = reinterpret_cast<int32_t*>(p); p += 256;
  w.Z = reinterpret_cast<double*>(p); p += al((size_t)n * nev * 8);
  w.tmp = reinterpret_cast<double2*>(p); p += al((size_t)NB * n * sizeof(double2));
  w.ybuf = reinterpret_cast<double2*>(p); p += al((size_t)2 * n * sizeof(double2));
  w.xbuf = reinterpret_cast<double2*>(p); p += al((size_t)2 * n * sizeof(double2));
  w.bar = reinterpret_cast<unsigned*>(p); p += al((size_t)TRI_BAR_WORDS * sizeof(unsigned));
  w.y2 = reinterpret_cast<double2*>(p); p += al((size_t)n * sizeof(double2));
  w.v2 = reinterpret_cast<double2*>(p); p += al((size_t)n * sizeof(double2));
  w.wev = reinterpret_cast<double*>(p); p += al((size_t)nev * 8);
  w.end = p;
  return w;
}

size_t hegv_work(int n, int nev) {
  static char probe alignas(256);
  return (size_t)(hegv_ws(&probe, n, nev).end - &probe);
}

// Launch shape of the resident tridiagonalisation: it takes the last m
// steps, m as large as the LDS of the device's compute units holds
// (c m double2 per workgroup, at most one workgroup per CU), aiming at
// TRI_CTARGET columns per workgroup; steps before n-1-m run as column
// launches.  A step of the resident kernel costs about as much as the two
// launches of a column step (grid barrier and the round trips of the
// published vectors; measured on MI355X: slower at n = 480, 11% faster at
// n = 1440), so problems below n = TRI_MIN_N keep column launches.
// k0 < 0: not used.
struct TriPlan {
  int k0 = -1, G = 0, c = 0;
  size_t lds = 0;
};
constexpr int TRI_CTARGET = 8;
constexpr int TRI_MIN_N = 1024;
int hegv_resident_min_n() { return TRI_MIN_N; }

static TriPlan tri_plan(int n) {
  TriPlan p;
  if (n < TRI_MIN_N) return p;
  int dev = 0, cus = 0, lds = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return p;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess)
    return p;
  if (!coop || cus <= 0 || lds <= 4096) return p;
  const size_t budget = (size_t)lds - 4096;  // static LDS of the kernel stays below 4 KB
  for (int m = std::min(n - 1, TRI_THREADS * TRI_RMAX); m >= 1; --m) {
    const int cfit = (int)std::min<size_t>(TRI_CMAX, budget / ((size_t)m * sizeof(double2)));
    if (cfit < 1) continue;
    int G = (int)ceil_div(m, std::min(cfit, TRI_CTARGET));
    if (G > cus) G = cus;
    const int c = (int)ceil_div(m, G);
    if (c > cfit) continue;
    p.k0 = n - 1 - m;
    p.G = G;
    p.c = c;
    p.lds = (size_t)c * m * sizeof(double2);
    return p;
  }
  return p;
}

int hegv(int n, int nev, double2* H, int ldh, double2* S, int lds_, double* w, double2* C, int ldc, void* work,
         int32_t* info, int32_t* ndead, hipStream_t s) {
  HegvWs ws = hegv_ws(work, n, nev);
  TimerScope ts(KF_HEGV, s);
  int rc;
  const bool deflate = ndead != nullptr;
  const PotrfWs pw = potrf_ws(ws.potrf, n);
  if ((rc = potrf_impl(n, S, lds_, ws.potrf, info, n, deflate, ndead, s))) return rc;
  // The two triangular solves of the reduction, Y = L^-1 H and
  // K = L^-1 Y^H, and the final C = L^-H Z go through X = L^-1: the blocked
  // solve runs once, on the identity (its result is exactly zero above the
  // diagonal), and each solve becomes one product, three launches instead
  // of three blocked solves of about 3n/32 launches each.
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)n * n, 256), 4096)),
                     dim3(256), 0, s, ws.X, n, n);
  KS_LAUNCH_CHECK("identity");
  if ((rc = trsm('N', n, n, S, lds_, ws.X, n, ws.potrf, ws.tmp, info, s, 0))) return rc;
  // Y = X H (in K's buffer), K = Y X^H (in H), then K <- (K + K^H)/2
  if ((rc = zgemm('N', 'N', n, n, n, 1.0, ws.X, n, H, ldh, 0.0, ws.K, n, s))) return rc;
  if ((rc = zgemm('N', 'C', n, n, n, 1.0, ws.K, n, ws.X, n, 0.0, H, ldh, s))) return rc;
  hipLaunchKernelGGL(k_hermitise_to, dim3((unsigned)n), dim3(256), 0, s, H, ldh, ws.K, n, n,
                     deflate ? pw.bound : nullptr);
  KS_LAUNCH_CHECK("hermitise");
  if (deflate) {
    hipLaunchKernelGGL(k_deflate_diag, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, ws.K, n, n, pw.dead,
                       pw.bound);
    KS_LAUNCH_CHECK("deflate_diag");
  }
  // Householder tridiagonalisation: one column per launch while the
  // trailing matrix is larger than the LDS of the device holds, then the
  // resident kernel for the remaining steps
  const TriPlan tp = tri_plan(n);
  const int klds = std::max(0, n - 1 - TAIL_MAX);  // first step of the LDS tail
  const int kres = tp.k0 >= 0 ? tp.k0 : klds;       // launches up to here
  // Trailing sizes above 512: two launches per column (product, then
  // update).  From 512 down, one launch per column after the first: the
  // update of step k fused with the product of step k+1, and a last update.
  auto column_steps = [&](int kbeg, int kend) {
    int k = kbeg;
    for (; k < kend && n - k - 1 > 512; ++k) {
      const int len = n - k - 1;
      hipLaunchKernelGGL(k_house_hemv, dim3((unsigned)ceil_div(len, 4)), dim3(256), 0, s, ws.K, n, n, k, ws.tau,
                         ws.d, ws.e, ws.v, ws.y);
      hipLaunchKernelGGL(k_her2, dim3((unsigned)ceil_div(len, 32), (unsigned)ceil_div(len, 32)), dim3(256), 0, s,
                         ws.K, n, n, k, ws.y, ws.tau, ws.v);
    }
    if (k >= kend) return;
    double2* vb[2] = {ws.v, ws.v2};
    double2* yb[2] = {ws.y, ws.y2};
    int p = 0;
    hipLaunchKernelGGL(k_house_hemv_reg<8>, dim3((unsigned)ceil_div(n - k - 1, 4)), dim3(256), 0, s, ws.K, n, n, k,
                       ws.tau, ws.d, ws.e, vb[p], yb[p]);
    for (; k + 1 < kend; ++k, p ^= 1) {
      const int len = n - k - 1;  // >= 2: k + 1 < kend <= n - 1
      hipLaunchKernelGGL(k_her2_house_hemv_reg<8>, dim3((unsigned)ceil_div(len - 1, 4)), dim3(256), 0, s, ws.K, n,
                         n, k, ws.tau, ws.d, ws.e, vb[p], yb[p], vb[p ^ 1], yb[p ^ 1]);
    }
    const int len = n - k - 1;
    hipLaunchKernelGGL(k_her2, dim3((unsigned)ceil_div(len, 32), (unsigned)ceil_div(len, 32)), dim3(256), 0, s,
                       ws.K, n, n, k, yb[p], ws.tau, vb[p]);
  };
  column_steps(0, kres);
  KS_LAUNCH_CHECK("tridiagonalisation");
  bool resident = false;
  if (tp.k0 >= 0) {
    hipLaunchKernelGGL(k_tri_reset, dim3(1), dim3(256), 0, s, ws.bar);
    KS_LAUNCH_CHECK("tridiagonalisation reset");
    double2* Kp = ws.K;
    int ldk = n, nn = n, k0 = tp.k0, c = tp.c;
    double2* taup = ws.tau;
    double* dp = ws.d;
    double* ep = ws.e;
    double2* yb = ws.ybuf;
    double2* xb = ws.xbuf;
    unsigned* bar = ws.bar;
    void* args[] = {&Kp, &ldk, &nn, &k0, &c, &taup, &dp, &ep, &yb, &xb, &bar, &info};
    const hipError_t le = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_tridiag_resident),
                                                     dim3((unsigned)tp.G), dim3(TRI_THREADS), args,
                                                     (unsigned)tp.lds, s);
    if (le == hipSuccess) {
      resident = true;
    } else {
      (void)hipGetLastError();  // not enqueued: continue one column per launch
    }
  }
  if (!resident) {
    // the last steps (trailing matrix of at most TAIL_MAX) in one workgroup
    const int kfrom = std::max(kres, klds);
    column_steps(kres, kfrom);
    KS_LAUNCH_CHECK("tridiagonalisation");
    if (n >= 2) {
      const int mt = n - kfrom - 1;
      const size_t lds = ((size_t)mt * mt + 4 * (size_t)mt) * sizeof(double2);
      hipLaunchKernelGGL(k_tridiag_tail_lds, dim3(1), dim3(TAIL_THREADS), lds, s, ws.K, n, n, kfrom, ws.tau, ws.d,
                         ws.e);
      KS_LAUNCH_CHECK("tridiagonalisation tail");
    } else {
      hipLaunchKernelGGL(k_tridiag_tail, dim3(1), dim3(64), 0, s, ws.K, n, n, ws.d, ws.e, ws.tau);
    }
  }
  // the deflating solve writes w directly; the strict one commits it at the
  // end only when the factorisation succeeded
  double* wout = deflate ? w : ws.wev;
  hipLaunchKernelGGL(k_bisect, dim3(nev), dim3(64), (size_t)2 * n * sizeof(double), s, ws.d, ws.e, n, nev, wout,
                     ws.tnorm);
  hipLaunchKernelGGL(k_clusters, dim3(1), dim3(64), 0, s, wout, nev, ws.tnorm, ws.cl, ws.ncl);
  hipLaunchKernelGGL(k_inverse_iteration, dim3(nev), dim3(256), (size_t)n * (5 * sizeof(double) + sizeof(int)), s,
                     ws.d, ws.e, n, wout, ws.tnorm, ws.cl, ws.ncl, ws.Z, n);
  KS_LAUNCH_CHECK("bisection / inverse iteration");
  // Q Z_T into H (no longer needed), then C = L^-H (Q Z_T) = X^H (Q Z_T)
  {
    const size_t lds = (size_t)n * sizeof(double2);
    const int need = (int)ceil_div(std::max(n - 1, 1), 64);  // reflector entries per lane
    if (need <= 8)
      hipLaunchKernelGGL(k_backtransform_reg<8>, dim3(nev), dim3(64), lds, s, ws.K, n, n, ws.tau, ws.Z, n, H, ldh);
    else if (need <= 16)
      hipLaunchKernelGGL(k_backtransform_reg<16>, dim3(nev), dim3(64), lds, s, ws.K, n, n, ws.tau, ws.Z, n, H, ldh);
    else if (need <= 24)
      hipLaunchKernelGGL(k_backtransform_reg<24>, dim3(nev), dim3(64), lds, s, ws.K, n, n, ws.tau, ws.Z, n, H, ldh);
    else if (need <= 48)
      hipLaunchKernelGGL(k_backtransform_reg<48>, dim3(nev), dim3(64), lds, s, ws.K, n, n, ws.tau, ws.Z, n, H, ldh);
    else
      hipLaunchKernelGGL(k_backtransform, dim3(nev), dim3(64), lds, s, ws.K, n, n, ws.tau, ws.Z, n, H, ldh);
    KS_LAUNCH_CHECK("backtransform");
  }
  if (deflate) return zgemm('C', 'N', n, nev, n, 1.0, ws.X, n, H, ldh, 0.0, C, ldc, s);
  // strict: C staged in K (free after the back-transform), then committed
  if ((rc = zgemm('C', 'N', n, nev, n, 1.0, ws.X, n, H, ldh, 0.0, ws.K, n, s))) return rc;
  hipLaunchKernelGGL(k_commit_results, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)n * nev, 256), 2048)),
                     dim3(256), 0, s, ws.wev, w, nev, ws.K, n, C, ldc, n, info);
  KS_LAUNCH_CHECK("commit");
  return 0;
}

// ---------------------------------------------------------------- reduction variants
// K = L^-1 H L^-H, three ways, for the comparison of the paper's choice (two
// triangular solves instead of a two-sided reduction) on the GPU:
//   0: L^-1 once (the blocked solve on the identity), then K = (L^-1 H) L^-H
//      as two products (the form the eigensolve uses);
//   1: the two triangular solves: Y = L^-1 H, then K = L^-1 Y^H (H Hermitian);
//   2: a blocked two-sided reduction of the HEGST type: for each diagonal
//      block, A11 <- L11^-1 A11 L11^-H, A21 <- A21 L11^-H - L21 A11 / 2,
//      A22 <- A22 - A21 L21^H - L21 A21^H, A21 <- A21 - L21 A11 / 2,
//      A21 <- L22^-1 A21 (the trailing blocks are reduced by the later
//      steps); the lower triangle holds K, the upper is set from it.
// Each ends with K <- (K + K^H)/2.

// B = A^H (n x n)
__global__ void k_conj_transpose(const double2* __restrict__ A, int lda, double2* __restrict__ B, int ldb, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double2 a = A[j + (int64_t)i * lda];
    B[i + (int64_t)j * ldb] = make_double2(a.x, -a.y);
  }
}

// upper triangle from the lower one: K_ij = conj(K_ji) for i < j
__global__ void k_upper_from_lower(double2* __restrict__ K, int ldk, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i < j) {
      const double2 a = K[j + (int64_t)i * ldk];
      K[i + (int64_t)j * ldk] = make_double2(a.x, -a.y);
    } else if (i == j) {
      K[i + (int64_t)j * ldk].y = 0.0;
    }
  }
}

static unsigned grid_nn(int n) { return (unsigned)std::min<int64_t>(ceil_div((int64_t)n * n, 256), 4096); }

int reduce_variant(int variant, int n, const double2* H, int ldh, double2* S, int lds_, double2* K, int ldk,
                   void* work, int32_t* info, hipStream_t s) {
  HegvWs ws = hegv_ws(work, n, 1);
  PotrfWs pw = potrf_ws(ws.potrf, n);
  int rc;
  if ((rc = potrf_impl(n, S, lds_, ws.potrf, info, n, false, nullptr, s))) return rc;
  const double2* L = S;
  if (variant == 0) {
    hipLaunchKernelGGL(k_set_identity, dim3(grid_nn(n)), dim3(256), 0, s, ws.X, n, n);
    if ((rc = trsm('N', n, n, L, lds_, ws.X, n, ws.potrf, ws.tmp, info, s, 0))) return rc;
    if ((rc = zgemm('N', 'N', n, n, n, 1.0, ws.X, n, H, ldh, 0.0, ws.K, n, s))) return rc;
    if ((rc = zgemm('N', 'C', n, n, n, 1.0, ws.K, n, ws.X, n, 0.0, K, ldk, s))) return rc;
  } else if (variant == 1) {
    if ((rc = copy_block(H, ldh, ws.X, n, n, n, s))) return rc;
    if ((rc = trsm('N', n, n, L, lds_, ws.X, n, ws.potrf, ws.tmp, info, s, 0))) return rc;
    hipLaunchKernelGGL(k_conj_transpose, dim3(grid_nn(n)), dim3(256), 0, s, ws.X, n, K, ldk, n);
    if ((rc = trsm('N', n, n, L, lds_, K, ldk, ws.potrf, ws.tmp, info, s, 0))) return rc;
  } else {
    if ((rc = copy_block(H, ldh, K, ldk, n, n, s))) return rc;
    for (int k0 = 0; k0 < n; k0 += NB) {
      const int kb = std::min(NB, n - k0);
      const int r0 = k0 + kb, rest = n - r0;
      const double2* linv = pw.linv + (size_t)(k0 / NB) * NB * NB;
      double2* A11 = K + k0 + (int64_t)k0 * ldk;
      // A11 <- L11^-1 A11 L11^-H
      if ((rc = zgemm('N', 'N', kb, kb, kb, 1.0, linv, NB, A11, ldk, 0.0, ws.K, n, s))) return rc;
      if ((rc = zgemm('N', 'C', kb, kb, kb, 1.0, ws.K, n, linv, NB, 0.0, A11, ldk, s))) return rc;
      if (rest <= 0) break;
      double2* A21 = K + r0 + (int64_t)k0 * ldk;
      double2* A22 = K + r0 + (int64_t)r0 * ldk;
      const double2* L21 = L + r0 + (int64_t)k0 * lds_;
      const double2* L22 = L + r0 + (int64_t)r0 * lds_;
      // A21 <- A21 L11^-H - L21 A11 / 2
      if ((rc = zgemm('N', 'C', rest, kb, kb, 1.0, A21, ldk, linv, NB, 0.0, ws.X, n, s))) return rc;
      if ((rc = zgemm('N', 'N', rest, kb, kb, -0.5, L21, lds_, A11, ldk, 1.0, ws.X, n, s))) return rc;
      // A22 <- A22 - A21 L21^H - L21 A21^H
      if ((rc = zgemm('N', 'C', rest, rest, kb, -1.0, ws.X, n, L21, lds_, 1.0, A22, ldk, s))) return rc;
      if ((rc = zgemm('N', 'C', rest, rest, kb, -1.0, L21, lds_, ws.X, n, 1.0, A22, ldk, s))) return rc;
      // A21 <- A21 - L21 A11 / 2, then L22^-1 A21
      if ((rc = zgemm('N', 'N', rest, kb, kb, -0.5, L21, lds_, A11, ldk, 1.0, ws.X, n, s))) return rc;
      if ((rc = trsm('N', rest, kb, L22, lds_, ws.X, n, ws.potrf, ws.tmp, info, s, r0 / NB))) return rc;
      if ((rc = copy_block(ws.X, n, A21, ldk, rest, kb, s))) return rc;
    }
    hipLaunchKernelGGL(k_upper_from_lower, dim3(grid_nn(n)), dim3(256), 0, s, K, ldk, n);
  }
  // K <- (K + K^H)/2 (out of place through X)
  hipLaunchKernelGGL(k_hermitise_to, dim3((unsigned)n), dim3(256), 0, s, K, ldk, ws.X, n, n, nullptr);
  if ((rc = copy_block(ws.X, n, K, ldk, n, n, s))) return rc;
  KS_LAUNCH_CHECK("reduce_variant");
  return 0;
}

}  // namespace ks
