// GEMM and dense-solver entry points shared between translation units.
#pragma once

#include <algorithm>

#include "ks_plan.hpp"

namespace ks {

// Up to three column segments of nb columns each, sharing ld: the LOBPCG
// basis V = [X W P] without copying it into one buffer.
template <typename T2>
struct BlockList {
  const T2* p[3];
  int64_t ld;
  int nb;
};

struct GramShape {
  int ntile, ntu, nsplit;
  int64_t kper;
};
// Launch shape for ntile x ntile tiles (upper triangle unless full) on a
// device with `slots` resident Gram workgroups.
GramShape gram_shape(int ntile, int64_t K, bool full, int slots);
// Partial-sum workspace for every Gram of at most m columns.
size_t gram_work_bytes(int m, int64_t K);

// S = A^H B1 (and H = A^H B2 when B2 != null) for the first m columns of the
// block lists, K rows; outputs Hermitian, FP64 complex, column-major.
template <typename T>
int gram(const BlockList<c2<T>>& A, const BlockList<c2<T>>& B1, const BlockList<c2<T>>* B2, int m, int64_t K,
         double2* S, int lds, double2* H, int ldh, void* work, hipStream_t s);

// G = A^H B (every tile, not Hermitian), FP64 complex column-major.
template <typename T>
int gram_general(const BlockList<c2<T>>& A, const BlockList<c2<T>>& B, int m, int64_t K, double2* G, int ldg,
                 void* work, hipStream_t s);

// out = V - X (X^H V) for nb-column blocks (cg.hip).  G: nb x nb FP64;
// Cbuf: nb x nb (or more) in the block precision; gram_ws: gram_work_bytes(nb, Ng).
template <typename T>
int project_out(const c2<T>* X, const c2<T>* V, c2<T>* out, int64_t ld, int nb, int64_t Ng, double2* G, void* Cbuf,
                void* gram_ws, hipStream_t s);

// out[b] = ||A[:, b]|| (Euclidean, FP64 sums in a fixed order); partial
// holds column_norms_partial(nb) doubles (cg.hip).
size_t column_norms_partial(int nb);
template <typename T>
int column_norms(const c2<T>* A, int64_t ld, int nb, int64_t Ng, double* partial, double* out, hipStream_t s);

// Y = V C; with Yp, Yp = V[:, pstart:m] C[pstart:m, :] as well.  Without
// Yp: upper = C is upper triangular (the zero part is skipped), and Yadd
// (may be Y) gives Y = Yadd + V C.
template <typename T>
int rotate(const BlockList<c2<T>>& V, int m, int pstart, const c2<T>* C, int ldc, int ncol, int64_t Ng, c2<T>* Y,
           c2<T>* Yp, int64_t ldy, hipStream_t s, bool upper = false, const c2<T>* Yadd = nullptr);

int zgemm(char ta, char tb, int M, int N, int K, double alpha, const double2* A, int lda, const double2* B,
          int ldb, double beta, double2* C, int ldc, hipStream_t s);

// ---- dense FP64 solver (dense.hip) ----
size_t hegv_work(int n, int nev);
// Largest order of the dense eigensolve: inverse iteration keeps five doubles
// and an int per row in LDS (44 bytes; 160 KB per workgroup).
constexpr int kHegvMaxN = 3700;
// Smallest n whose tridiagonalisation uses the resident (cooperative) kernel;
// only that kernel can report info = -1.
int hegv_resident_min_n();
// ndead == nullptr: strict solve (info = n + k on a failed Cholesky, and then
// w and C are left unchanged).  Otherwise the Cholesky deflates: basis
// vectors that depend numerically on earlier ones are dropped (zero rows of
// C), their count added to *ndead, and info only reports the resident
// tridiagonalisation's barrier (-1).
int hegv(int n, int nev, double2* H, int ldh, double2* S, int lds, double* w, double2* C, int ldc, void* work,
         int32_t* info, int32_t* ndead, hipStream_t s);
// Cholesky S = L L^H in place (lower), info as for hegv (k, not n + k).
size_t potrf_work(int n);
int potrf(int n, double2* S, int lds, void* work, int32_t* info, hipStream_t s);
// The same with deflation of dependent columns (pivot 1, zero column below
// it, zero row in the inverted diagonal block), counted in *ndead.
int potrf_deflate(int n, double2* S, int lds, void* work, int32_t* info, int32_t* ndead, hipStream_t s);
// B <- op(L)^-1 B for the lower factor L from potrf (its workspace holds
// the inverted diagonal blocks); op 'N' or 'C'.
int trsm(char op, int n, int ncol, const double2* L, int ldl, double2* B, int ldb, void* potrf_ws, void* tmp,
         const int32_t* info, hipStream_t s, int blk0 = 0);
// K = L^-1 H L^-H after the Cholesky S = L L^H (S overwritten by L; info as
// hegv), by variant 0 (L^-1 and two products), 1 (two triangular solves) or
// 2 (blocked two-sided reduction); workspace hegv_work(n, 1).
int reduce_variant(int variant, int n, const double2* H, int ldh, double2* S, int lds, double2* K, int ldk,
                   void* work, int32_t* info, hipStream_t s);
// The real-symmetric form of reduce_variant (dense_real.hip): S = L L^T,
// K = L^-1 H L^-T, real FP64; workspace real_reduce_work(n).
size_t real_reduce_work(int n);
int real_reduce_variant(int variant, int n, const double* H, int ldh, double* S, int lds, double* K, int ldk,
                        void* work, int32_t* info, hipStream_t s);

}  // namespace ks
