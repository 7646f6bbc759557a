/*
 * ksh.h - C ABI of an MI355X-native LOBPCG eigensolver for real-space
 * Kohn-Sham DFT (the SCF hot path of arXiv 2512.04447).
 *
 * The paper names four per-SCF-iteration tasks (the task-list paragraph):
 * (1) FFTs that apply the Laplacian to every orbital in one batched call,
 * (2) the dense products that form the LOBPCG subspace matrices H and S,
 * (3) the generalised Hermitian eigensolve H X = lambda S X, reduced by a
 *     Cholesky factor S = L L^H to K Z = lambda Z, K = L^-1 H L^-H (Eq. 1),
 *     with K formed by two triangular solves (paragraph after Eq. 1), and
 * (4) the separable nonlocal pseudopotential operator.
 * Everything behind this header is hand-written HIP for gfx950.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: Hartree atomic units (Ha, bohr).
 * Grid: orthorhombic, n[0] x n[1] x n[2] points; point (i,j,k) sits at
 *   (i L0/n0, j L1/n1, k L2/n2); its linear index is (i*n1 + j)*n2 + k.
 *   Ng = n0*n1*n2.  Each n must factor into 2, 3, 5 and 7.
 * Transforms: forward sum_r exp(-i G.r) f(r), inverse exp(+i G.r)/Ng,
 *   G = 2 pi m / L per axis with m wrapped into [-n/2, n/2); T(G) = |G|^2/2.
 * Blocks: an orbital block of nb columns is column-major, column (band) j
 *   starting at base + j*ld elements, ld >= Ng, interleaved complex:
 *   double2 (complex128) for KS_FP64 plans, float2 (complex64) for the
 *   mixed-precision plans.
 * Pointers: unless stated otherwise, data pointers are DEVICE pointers owned
 *   by the caller; the library never frees them.  Plan-owned tables live in
 *   device memory allocated by ks_plan_create and freed by ks_plan_destroy.
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls are
 *   stream ordered; a call returns once its work is enqueued, except where
 *   noted (ks_plan_create; lobpcg_init and lobpcg_step when given a host
 *   summary buffer, which they fill with one copy and wait for).
 * Errors: every function returns 0 on success; -i when argument i (1-based)
 *   is invalid (checked on the host before any launch); KS_E_HIP - code for
 *   a HIP runtime error; KS_E_WORKSPACE when work_bytes is too small;
 *   KS_E_NUMERIC when a numerical breakdown stops the computation.  The
 *   message of the last error on the calling thread is ks_last_error().
 * Concurrency: one plan is used by one stream at a time.
 */
#ifndef KSH_H
#define KSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KS_E_HIP (-1000)
#define KS_E_WORKSPACE (-2001)
#define KS_E_NUMERIC (-2002)
#define KS_E_UNSUPPORTED (-2003)

/* Arithmetic of a plan.
 * KS_FP64: blocks complex128; FFT, H-apply, Gram, rotation and subspace
 *   solve all in FP64.
 * KS_MIXED_FP32: blocks complex64; FFT and H-apply in FP32; Gram products in
 *   FP32 with FP32 accumulation inside each K chunk and FP64 summation of
 *   the chunks; Cholesky, triangular solves, eigensolve and the X
 *   re-orthonormalisation factor in FP64; rotation in FP32.
 * KS_MIXED_BF16X3: reserved for an H Gram from three bf16 products
 *   (hi*hi + hi*lo + lo*hi) per real product; not built: ks_plan_create
 *   returns KS_E_UNSUPPORTED for it. */
typedef enum { KS_FP64 = 0, KS_MIXED_FP32 = 1, KS_MIXED_BF16X3 = 2 } ks_precision;

typedef struct {
  int32_t n[3];
  double L[3];
} ks_grid;

/* Separable (Kleinman-Bylander) projector set, task (4) of the task list.
 * HOST pointers, read once by ks_plan_create.
 * Atom a owns support points supp_idx[atom_supp_ptr[a] .. atom_supp_ptr[a+1])
 * (grid linear indices) and projectors atom_proj_ptr[a] .. atom_proj_ptr[a+1].
 * The values of its projector j (0-based within the atom) at its support
 * points are beta[beta_ptr[a] + j*|S_a| + s].  D[p] is the coupling of
 * projector p (Ha).  The operator is sum_p b_p D_p b_p^T (real b_p). */
typedef struct {
  int32_t n_atoms;
  int32_t n_proj;
  int64_t n_supp;
  const int32_t* atom_supp_ptr; /* n_atoms + 1 */
  const int32_t* supp_idx;      /* n_supp */
  const int32_t* atom_proj_ptr; /* n_atoms + 1 */
  const int64_t* beta_ptr;      /* n_atoms + 1 */
  const double* beta;           /* beta_ptr[n_atoms] */
  const double* D;              /* n_proj */
} ks_projset;

typedef struct ks_plan ks_plan;

/* LOBPCG iteration state (Knyazev's [X, W, P] Rayleigh-Ritz; the paper's
 * eigensolver).  All block pointers are device blocks of plan->nb_max or
 * fewer columns with the common leading dimension ld.  X, AX (= H X), P, AP,
 * W, AW hold the iterate; Xn, Pn and T1 are scratch blocks of the same
 * shape.  lobpcg_step swaps the pointer pairs (X,Xn), (P,Pn) and (W,Xn) as
 * it goes: read them back after each call.  theta[nb] (Ritz values) and
 * res[nb] (residual 2-norms of the block the step started from) are device
 * arrays of doubles; status is a device array of KS_STATUS_WORDS int32.
 * host_summary (optional, host memory of 16*nb + 4*KS_STATUS_WORDS bytes,
 * pinned for an asynchronous copy): when set, lobpcg_init and lobpcg_step
 * end with one device-to-host copy of theta[nb], res[nb] (doubles) and the
 * status words into it and wait for that copy; when NULL they never
 * synchronise the stream. */
typedef struct {
  int32_t nb;
  int32_t has_p;   /* 0 before the first step; set by lobpcg_step */
  int64_t ld;
  void* X;
  void* AX;
  void* W;
  void* AW;
  void* P;
  void* AP;
  void* Xn;
  void* Pn;
  void* T1;
  double* theta;
  double* res;
  int32_t* status;
  void* host_summary;
  int32_t iter;    /* iterations done */
  /* 1 once lobpcg_step has left the next step's P Gram in p_gram; cleared
   * by lobpcg_init.  A caller that replaces P (or the state) between steps
   * sets it to 0. */
  int32_t p_gram_ok;
  /* Optional device array of nb*nb complex128 values (16*nb*nb bytes,
   * column-major) that carries the Gram matrix of the next step's P from
   * one lobpcg_step to the next: the step's P = V_[W P] C_[W P], so
   * P^H P = C_[W P]^H S_[W P] C_[W P] is formed from the step's own
   * subspace matrices (two products of its m - nb square block) instead of
   * a pass over P's Ng rows.  The next step uses it when p_gram_ok is set.
   * FP64 plans only (a mixed plan's P, rotated in FP32, departs from that
   * product by the FP32 rounding); NULL, or a mixed plan: every step forms
   * P's Gram from P itself. */
  void* p_gram;
} ks_lobpcg_state;

/* Status words written by every lobpcg_init / lobpcg_step (cleared at its
 * start).  Deflation: a column that depends numerically on the columns
 * before it (Cholesky pivot not above 1e-14 of the largest diagonal entry)
 * is dropped instead of stopping the iteration: in W or P it becomes an
 * exactly-zero column, in the basis [X W P] it gets zero Ritz coefficients. */
#define KS_STATUS_WORDS 8
#define KS_ST_FLAGS 0      /* KS_FLAG_* bits */
#define KS_ST_DEAD_W 1     /* W columns deflated by its orthonormalisation */
#define KS_ST_DEAD_P 2     /* P columns deflated likewise */
#define KS_ST_DEAD_BASIS 3 /* basis vectors dropped by the subspace Cholesky */
#define KS_ST_DEAD_X 4     /* X columns deflated (initial Cholesky-QR, mixed re-orthonormalisation) */
#define KS_ST_INFO 5       /* 0, or -1: the resident tridiagonalisation's grid barrier timed out */
#define KS_FLAG_DEFLATED 1     /* some column was deflated (the step is still valid) */
#define KS_FLAG_SOLVE_FAILED 2 /* KS_ST_INFO != 0: theta and the new block are not valid */
#define KS_FLAG_NONFINITE 4    /* a Ritz value or residual norm is not finite */

/* Preconditioner kinds.  KS_PRECOND_CNN applies the learned network below to
 * each residual (input channels Re r~, Im r~, h^2 (V_loc - theta_i), with
 * r~ = r sqrt(Ng)/||r|| and h = L0/n0; output w = y0 + i y1).
 * KS_PRECOND_CNN_TPA applies it to the Teter-Payne-Allan output p = K_TPA(r)
 * instead and adds its input: w = (p~0 + y0) + i (p~1 + y1), p~ = p sqrt(Ng)/
 * ||p|| (a network whose last layer is zero reproduces TPA).  Either kind
 * keeps the band's unlearned column (r, or p) where the network output is
 * not finite. */
#define KS_PRECOND_NONE 0
#define KS_PRECOND_TPA 1
#define KS_PRECOND_CNN 2
#define KS_PRECOND_CNN_TPA 3

typedef struct ks_lobpcg_opts {
  int32_t precond;  /* KS_PRECOND_* */
  int32_t pad_;
  /* Soft locking: a band with residual norm <= lock_tol contributes an
   * exactly-zero column to W and P (its X column stays). */
  double lock_tol;
  const float* cnn_params; /* device, KS_CNN_NPARAM floats; the CNN kinds only */
} ks_lobpcg_opts;

/* Learned preconditioner: three periodic 3x3x3 convolutions 3 -> 16 -> 16 -> 2
 * with bias and SiLU between them (no activation after the last).  Parameter
 * vector (FP32): w1[16][3][27], b1[16], w2[16][16][27], b2[16], w3[2][16][27],
 * b3[2], with w[o][i][(dx+1)*9 + (dy+1)*3 + dz+1] weighting in[i](x+dx, y+dy,
 * z+dz) (cross-correlation, periodic).  Activations FP32, layout
 * [sample][channel][Ng]. */
#define KS_CNN_NPARAM 9106

/* Which operation a workspace query is for (KS_OP_PRECOND: ks_precond_apply
 * with KS_PRECOND_NONE or KS_PRECOND_TPA; KS_OP_PRECOND_CNN: with the
 * learned kinds). */
#define KS_OP_APPLY_H 1
#define KS_OP_PRECOND 2
#define KS_OP_LOBPCG 3
#define KS_OP_PRECOND_CNN 5

/* Build a plan: radix schedules and twiddle tables for the three axes, the
 * projector tables in device memory (values in the plan's precision) plus
 * their inverse by grid point (for the deterministic scatter), and launch
 * configurations.  `proj` may be NULL or have n_proj == 0 (no nonlocal
 * term).  nb_max bounds the block width of later calls (at most 1233: the
 * subspace problem has order 3 nb_max, see hegv_reduce_solve).  Allocates device
 * memory; synchronises `stream` once at the end. */
int ks_plan_create(ks_plan** out, const ks_grid* grid, const ks_projset* proj,
                   int32_t nb_max, int32_t precision, void* stream);

/* A plan for the periodic part u of Bloch orbitals psi = exp(i k.r) u at a
 * Bloch vector k (the k-point variant of the same iteration; k = 0 gives
 * the plan of ks_plan_create).  Every entry point then applies
 * H_k = exp(-i k.r) H exp(i k.r): kinetic energy |G + k|^2 / 2 in the
 * FFT passes (the TPA preconditioner and the kinetic energies use it too;
 * the Hartree solve of ks_hartree does not), the local potential unchanged,
 * and the projectors seen by u at support point s of an atom
 * b_j(s) exp(-i k.d_s), d_s the displacement of the point from the atom
 * (the image nearest the atom), so that
 *   V_NL u = sum_j b_j exp(-i k.d) D_j <b_j exp(-i k.d) | u>.
 * kvec: host, 3 doubles, Cartesian (1/bohr).  supp_disp: host, 3 * n_supp
 * doubles (x, y, z of d_s in bohr, in the order of supp_idx), read once;
 * required when k != 0 and the set has projectors.  Internally each
 * projector becomes the real pair b cos(k.d), b sin(k.d), so an atom may
 * carry at most 4 projectors (s and p; KS_E_UNSUPPORTED otherwise). */
int ks_plan_create_k(ks_plan** out, const ks_grid* grid, const double* kvec, const ks_projset* proj,
                     const double* supp_disp, int32_t nb_max, int32_t precision, void* stream);
int ks_plan_destroy(ks_plan* plan);

/* Bytes of caller workspace that `op` needs for blocks of nb columns. */
int ks_workspace_size(const ks_plan* plan, int32_t op, int32_t nb, size_t* bytes);

/* Kohn-Sham H-apply (tasks (1) and (4) of the task list plus the local
 * potential):  hpsi = T psi + V_loc .* psi + sum_p b_p D_p (b_p^T psi).
 * v_loc: Ng reals (double for KS_FP64, float otherwise).  psi and hpsi must
 * not overlap.  T is applied by a batched 3D FFT over all nb columns. */
int ks_apply_h(const ks_plan* plan, const void* v_loc, const void* psi, int64_t ld_psi,
               void* hpsi, int64_t ld_hpsi, int32_t nb, void* work, size_t work_bytes,
               void* stream);

/* Residual and preconditioner (the preconditioned residuals are the W block
 * of LOBPCG):  R = AX - X diag(theta);  res[i] = ||r_i||_2;  W = K(R) with
 * K chosen by opts->precond:
 *   KS_PRECOND_NONE: the identity;
 *   KS_PRECOND_TPA: the Teter-Payne-Allan kinetic preconditioner,
 *     w_i = IFFT(K(x) FFT(r_i)), x = T(G)/E_i, E_i = <x_i|T|x_i>,
 *     K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4);
 *   KS_PRECOND_CNN / KS_PRECOND_CNN_TPA: the learned network (below) with
 *     parameters opts->cnn_params (device, KS_CNN_NPARAM floats) on r, or on
 *     the TPA output with its skip connection.
 * Columns with res[i] <= opts->lock_tol are written as zeros.  v_loc: Ng
 * reals of the plan's precision (the network's third input channel; may be
 * NULL for NONE and TPA).  All
 * blocks share ld.  Workspace: ks_workspace_size(KS_OP_PRECOND) for NONE and
 * TPA, ks_workspace_size(KS_OP_PRECOND_CNN) for the learned kinds. */
int ks_precond_apply(const ks_plan* plan, const ks_lobpcg_opts* opts, const void* v_loc, const void* X,
                     const void* AX, const double* theta, int64_t ld, int32_t nb, void* W, double* res, void* work,
                     size_t work_bytes, void* stream);

/* Generalised Hermitian eigensolve by the paper's reduction (Eq. 1 and the
 * paragraph after it), FP64 complex, column-major:
 *   L = chol(S) (lower);  Y = L^-1 H;  K = L^-1 Y^H (= L^-1 H L^-H);
 *   K <- (K + K^H)/2;  K = Q T Q^H (Householder);  lowest nev eigenpairs of
 *   the real tridiagonal T by bisection and inverse iteration;  Z = Q Z_T;
 *   C = L^-H Z.
 * On return w[0..nev) ascending, C (n x nev, ldc) with C^H S C = I, S holds
 * L in its lower triangle and H is overwritten.  info_dev (device int32):
 * 0 ok; n + k if the leading minor k of S is not positive definite (pivot
 * <= 1e-14 * max diag(S)); -1 if the grid barrier of the resident
 * tridiagonalisation (n >= 1024, one cooperative launch, co-residency
 * guaranteed by the runtime) gave up after its bounded wait.  When info is
 * not 0, w and C are left unchanged (the work after the factorisation still
 * runs on the device, on values that are then discarded).  n <= 3700
 * (inverse iteration keeps 44 bytes per row in LDS), so ks_plan_create
 * accepts nb_max <= 1233. */
int hegv_reduce_solve(int32_t n, int32_t nev, void* H, int32_t ldh, void* S, int32_t lds,
                      double* w, void* C, int32_t ldc, void* work, size_t work_bytes,
                      int32_t* info_dev, void* stream);
int hegv_workspace_size(int32_t n, int32_t nev, size_t* bytes);

/* The reduction step of the generalised eigensolve alone, by one of three
 * methods (the comparison behind the paper's choice of two triangular solves
 * over a two-sided reduction, paragraph after Eq. 1 and its eigensolver
 * figure): S = L L^H (lower, in place; info_dev as hegv_reduce_solve), then
 * K = L^-1 H L^-H, Hermitised, into K (n x n, ldk; H is not modified):
 *   KS_REDUCE_INVERSE: L^-1 by one blocked solve on the identity, then two
 *     products (what hegv_reduce_solve uses);
 *   KS_REDUCE_TWO_TRSM: Y = L^-1 H and K = L^-1 Y^H by two blocked
 *     triangular solves;
 *   KS_REDUCE_TWO_SIDED: a blocked two-sided reduction of the xHEGST type
 *     (per 32-column block: the diagonal block two-sided, the panel by one
 *     solve and two products, the trailing matrix by a rank-2k update).
 * Workspace: hegv_workspace_size(n, 1). */
#define KS_REDUCE_INVERSE 0
#define KS_REDUCE_TWO_TRSM 1
#define KS_REDUCE_TWO_SIDED 2
int hegv_reduce_variant(int32_t variant, int32_t n, const void* H, int32_t ldh, void* S, int32_t lds, void* K,
                        int32_t ldk, void* work, size_t work_bytes, int32_t* info_dev, void* stream);

/* The same three reductions for real symmetric H and S (the Gamma-point
 * case, where orbitals and subspace matrices are real: the real-versus-
 * complex comparison of the paper's eigensolver figure).  H, S, K: n x n
 * real FP64, column-major, device; S <- L (lower, in place; the strict
 * upper triangle does not enter the result and is left undefined), H is not modified, K receives
 * L^-1 H L^-T symmetrised.  info_dev (device int32): 0, or n + k when the
 * leading minor k of S is not positive definite (pivot <= 1e-14 max diag(S));
 * K is then meaningless.  Workspace: sygv_reduce_workspace_size(n)
 * (about 2 n^2 doubles).  Errors: -i for argument i before any launch. */
int sygv_reduce_variant(int32_t variant, int32_t n, const double* H, int32_t ldh, double* S, int32_t lds,
                        double* K, int32_t ldk, void* work, size_t work_bytes, int32_t* info_dev, void* stream);
int sygv_reduce_workspace_size(int32_t n, size_t* bytes);

/* hegv_reduce_solve for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and the same results, with the workspace taken from a
 * static device array of KS_NOALLOC_SCRATCH_BYTES (32 MiB) that each GPU the
 * library runs on holds until the process ends.  n <= KS_NOALLOC_MAX_N
 * (512); larger n (or a workspace beyond the array) returns -1 or
 * KS_E_WORKSPACE without launching anything.  Calls no hipMalloc or hipFree;
 * its kernels are never timed.  All calls on one GPU share that array:
 * calls that overlap on one GPU (different streams or threads) race and
 * give wrong results; serialise them. */
#define KS_NOALLOC_MAX_N 512
#define KS_NOALLOC_SCRATCH_BYTES (32u << 20)
#define KS_NOALLOC_MAX_DEVICES 64
int hegv_reduce_solve_noalloc(int32_t n, int32_t nev, void* H, int32_t ldh, void* S, int32_t lds, double* w, void* C,
                              int32_t ldc, int32_t* info_dev, void* stream);

/* LOBPCG start: X <- X L^-H with L = chol(X^H X) (Cholesky-QR of the initial
 * block in st->X), AX = H X, Rayleigh-Ritz on span(X): X <- X Z, then
 * AX = H X by a fresh H-apply; theta = Ritz values ascending.  Sets
 * st->has_p = 0, st->iter = 0 and the status words (res is not written). */
int lobpcg_init(const ks_plan* plan, const void* v_loc, ks_lobpcg_state* st, void* work,
                size_t work_bytes, void* stream);

/* One LOBPCG iteration, as the oracle's reading of Knyazev's method:
 *   1. R = AX - X Theta, res = column norms of R;  W = K(R) (ks_precond_apply
 *      with opts), zero for soft-locked bands (res <= lock_tol);
 *   2. W <- W - X (X^H W), then W <- W D L^-H (unit columns, Cholesky-QR
 *      within the block, deflating);
 *   3. AW = H W;
 *   4. (from the second step) P masked by the lock test, orthonormalised as
 *      W (its Gram from the previous step's subspace matrices when
 *      st->p_gram is set), AP = H P;
 *   5. S = V^H V, H = V^H AV for V = [X W P] (or [X W]), Hermitised; exactly
 *      zero columns decoupled (S_kk = 1, H_kk = 2 max|H_ii| + 1);
 *   6. lowest nb eigenpairs of H C = S C Theta by the reduction of
 *      hegv_reduce_solve with a deflating Cholesky (numerically dependent
 *      basis vectors get zero coefficients);
 *   7. X <- V C, P <- V_{[W P]} C_{[W P]};
 *   8. mixed plans: X <- X L^-H (Cholesky-QR, FP64 factor);
 *   9. AX = H X by a fresh H-apply (AP is formed afresh in the next step).
 * Status words as above; no host synchronisation unless st->host_summary
 * is set. */
int lobpcg_step(const ks_plan* plan, const void* v_loc, ks_lobpcg_state* st,
                const ks_lobpcg_opts* opts, void* work, size_t work_bytes, void* stream);

/* Convergence check by subspace angles: the sine of the largest principal
 * angle between the column spans of A and B (k orthonormal columns each,
 * the plan's precision, leading dimension ld),
 *   sin_max = sqrt(1 - sigma_min(A^H B)^2),
 * with A^H B from the Gram kernel and sigma_min^2 the lowest eigenvalue of
 * (A^H B)^H (A^H B) from the dense eigensolve (accurate to about 1e-7 in
 * sin_max).  Written to the device double *sin_max (NaN if the eigensolve
 * reports a failure).  k <= nb_max.  Workspace: ks_workspace_size(KS_OP_ANGLE, k). */
#define KS_OP_ANGLE 6
int ks_subspace_sin(const ks_plan* plan, const void* A, const void* B, int64_t ld, int32_t k, double* sin_max,
                    void* work, size_t work_bytes, void* stream);

/* The dense products of the path as building blocks (also what the GEMM
 * sweeps time): complex blocks of K rows (column-major, leading dimension
 * ld), complex128 for precision KS_FP64 and complex64 for KS_MIXED_FP32.
 * ks_gram_general: G = A^H B, m x m FP64 complex column-major (ldg >= m),
 * every tile computed (not Hermitised), products on the matrix cores
 * (FP64, or FP32 with FP64 sums of the K chunks).  Workspace:
 * ks_gram_workspace_size.  ks_rotate_block: Y = V C, V of m columns, C an
 * m x ncol matrix of the block precision (ldc >= m), Y of ncol columns
 * (ldy >= K); Y must not overlap V. */
int ks_gram_workspace_size(int64_t K, int32_t m, size_t* bytes);
int ks_gram_general(int32_t precision, int64_t K, int32_t m, const void* A, const void* B, int64_t ld, void* G,
                    int32_t ldg, void* work, size_t work_bytes, void* stream);
int ks_rotate_block(int32_t precision, int64_t K, int32_t m, const void* V, int64_t ld, const void* C, int32_t ldc,
                    int32_t ncol, void* Y, int64_t ldy, void* stream);

/* The self-consistent loop's steps around the eigensolve (the "Others" of
 * the paper's SCF cost breakdown), for plans of either precision; fields
 * are Ng FP64 values on the plan's grid.
 * ks_density: n(r) = sum_{i < nocc} f_i |x_i(r)|^2, electrons per grid point
 *   (sum_r n = sum_i f_i for orthonormal columns), from nocc columns of X
 *   (ld); occ: device array of nocc occupations, or NULL for 2 each.
 * ks_hartree: V_H from the periodic Poisson equation for rho = n / dV
 *   (dV = L0 L1 L2 / Ng): V_H(G) = 4 pi rho(G) / |G|^2, V_H(0) = 0 (uniform
 *   neutralising background), on the plan's FFT passes.
 * ks_lda_xc: exchange-correlation potential v_xc and energy per electron
 *   e_xc (may be NULL) of the local density approximation: Slater exchange
 *   and the Perdew-Zunger parametrisation of the Ceperley-Alder correlation;
 *   zero where rho <= 1e-30.
 * ks_scf_potential: v_eff = v_ion + V_H[n] + v_xc[n] (Ng reals in the
 *   plan's precision, ready for ks_apply_h and lobpcg_step) and terms[4] =
 *   (sum V_H n, sum v_xc n, sum e_xc n, sum n) on the device.
 * ks_mix_density: n_next = (1 - alpha) n_in + alpha n_out and
 *   resid[0] = ||n_out - n_in||_2 on the device.
 * Workspace (ks_hartree, ks_scf_potential, ks_mix_density):
 * ks_workspace_size(KS_OP_SCF, 1). */
#define KS_OP_SCF 7
int ks_density(const ks_plan* plan, const void* X, int64_t ld, int32_t nocc, const double* occ, double* n,
               void* stream);
int ks_hartree(const ks_plan* plan, const double* n, double* v_h, void* work, size_t work_bytes, void* stream);
int ks_lda_xc(const ks_plan* plan, const double* n, double* v_xc, double* e_xc, void* stream);
int ks_scf_potential(const ks_plan* plan, const double* n, const double* v_ion, void* v_eff, double* terms,
                     void* work, size_t work_bytes, void* stream);
int ks_mix_density(const ks_plan* plan, double alpha, const double* n_in, const double* n_out, double* n_next,
                   double* resid, void* work, size_t work_bytes, void* stream);

/* Training targets for the learned preconditioner: for every column i at
 * once, solve the Jacobi-Davidson correction equation
 *   P (H - theta_i) P t_i = P r_i,  P = I - X X^H,  t_i in range(P)
 * by conjugate gradients (X: nb orthonormal columns, e.g. the current Ritz
 * block; R: right-hand sides; T: output; all with leading dimension ld).
 * A column stops when ||residual|| <= rtol ||P r_i|| or its curvature
 * p^H A p is not positive.  iters[i] (device int32) receives the iterations
 * used, negated for a curvature stop.  Reads a 4-byte count back every 16
 * iterations to stop early.  Workspace: ks_workspace_size(KS_OP_JD). */
#define KS_OP_JD 4
int ks_jd_correction(const ks_plan* plan, const void* v_loc, const void* X, const double* theta,
                     const void* R, int64_t ld, int32_t nb, int32_t maxit, double rtol, void* T,
                     int32_t* iters, void* work, size_t work_bytes, void* stream);

/* Learned-preconditioner training kernels.  Every convolution (forward,
 * backward-data, weight gradient) runs on the bfloat16 matrix cores: its two
 * operands are rounded to the nearest bfloat16 (ties to even), products and
 * sums are FP32; parameters, activations, bias gradients and Adam are FP32,
 * sums over tiles and samples FP64.  cnn_workspace_size: floats of forward activations kept
 * for backward (act_floats) and bytes of backward workspace for nbatch
 * samples on the plan's grid. */
int cnn_workspace_size(const ks_plan* plan, int32_t nbatch, size_t* act_floats, size_t* work_bytes);
/* y[nbatch][2][Ng] = net(x[nbatch][3][Ng]); acts receives the activations. */
int cnn_forward(const ks_plan* plan, const float* params, int32_t nbatch, const float* x, float* y,
                float* acts, void* stream);
/* grads[KS_CNN_NPARAM] = dL/dparams given gy = dL/dy (overwritten, not
 * accumulated); sums over samples and grid points in a fixed order. */
int cnn_backward(const ks_plan* plan, const float* params, int32_t nbatch, const float* x,
                 const float* acts, const float* gy, float* grads, void* work, size_t work_bytes,
                 void* stream);
/* Scale-invariant loss per sample, loss[b] = ||y_b/|y_b| - t_b/|t_b| ||^2,
 * and gy = d(mean_b loss_b)/dy.  sums: 3*nbatch doubles of scratch. */
int cnn_loss(int32_t nbatch, int64_t Ng, const float* y, const float* t, float* gy, double* loss,
             double* sums, void* stream);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8); t >= 1. */
int cnn_adam_step(float* params, const float* grads, float* m, float* v, int32_t nparam, int32_t t,
                  float lr, void* stream);
/* Network input x[nb][3][Ng] from residual columns R (ld), their norms
 * rnorm[nb], v_loc and theta[nb].  rnorm may be NULL: each column is then
 * scaled by its own Euclidean norm, computed here (a zero column stays zero). */
int cnn_make_input(const ks_plan* plan, const void* R, int64_t ld, const double* rnorm,
                   const void* v_loc, const double* theta, int32_t nb, float* x, void* stream);
/* Skip connection of the residual network: y[b][c][:] += x[b][c][:] for the
 * first two channels (c = 0, 1) of nbatch samples on the plan's grid.  The
 * gradient with respect to the network output equals the one with respect
 * to y, so cnn_backward is unchanged. */
int cnn_add_skip(const ks_plan* plan, int32_t nbatch, const float* x, float* y, void* stream);
/* Inference of the network as lobpcg_step applies it (KS_PRECOND_CNN and
 * KS_PRECOND_CNN_TPA): y[nbatch][2][Ng] = net(x[nbatch][3][Ng]), every
 * layer on the bfloat16 matrix cores exactly as in cnn_forward.  buf: 32 * nbatch * Ng floats of scratch (the
 * act_floats of cnn_workspace_size suffice). */
int cnn_infer(const ks_plan* plan, const float* params, int32_t nbatch, const float* x, float* y,
              float* buf, void* stream);
/* One periodic 3x3x3 convolution 16 -> 16 channels on the bfloat16 matrix
 * cores: y[b][o][r] = bias[o] + sum_{i, d} w[o][i][d] x[b][i][r + d] (w as
 * in the parameter vector, [o][i][dx][dy][dz]; d in {-1, 0, 1}^3), with x
 * and w rounded to the nearest bfloat16 (ties to even), products and sums in
 * FP32, then SiLU when silu != 0.  x, y: nbatch x 16 x Ng floats, no
 * aliasing. */
int cnn_conv16_bf16(const ks_plan* plan, int32_t nbatch, const float* x, const float* w,
                    const float* b, int32_t silu, float* y, void* stream);

/* Kernel timing for measurement (not needed to solve anything).
 * ks_kernel_timer(1, id) starts recording a HIP event pair around every
 * later launch of kernel family `id` on the stream it is launched on;
 * ks_kernel_timer(0, id) stops recording.  ks_kernel_timer_read waits for
 * the recorded events, returns the summed kernel time (ms) and launch count
 * since the last start, and releases the events.  Families:
 * 0 Gram GEMM (every Gram), 1 rotation GEMM, 2 FFT pass A, 3 FFT pass B,
 * 4 FFT pass C, 5 nonlocal projection, 6 subspace solve (hegv as a whole),
 * 7 small GEMM, 8 the basis Gram of lobpcg_step alone (S and H of [X W P],
 * also counted in 0), 9 nonlocal scatter.
 * Host-side state shared by all threads; not for concurrent use. */
#define KS_KERNEL_FAMILIES 10
int ks_kernel_timer(int32_t enable, int32_t family);
int ks_kernel_timer_read(int32_t family, double* total_ms, int64_t* launches);

/* Thread-local message of the last failing call ("" if none). */
const char* ks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KSH_H */
