// Internal plan structure and the launch functions shared between the
// translation units of the ksh library.
#pragma once

#include <vector>

#include "ks_common.hpp"

namespace ks {

// Points per block of the nonlocal scatter (its projector lists are built
// for blocks of this many consecutive grid points).
constexpr int kScatterPts = 256;

constexpr int kMaxStages = 10;
constexpr int kThreads = 256;

// Radix schedule of one axis for the Stockham passes.
struct AxisPlan {
  int n;
  int nst;
  int rad[kMaxStages];
};

struct Fft3 {
  AxisPlan ax[3];
  double twopi_over_L[3];
  double kvec[3];  // Bloch vector (Cartesian, 1/bohr): kinetic |G + k|^2 / 2
  // H-applies of the LOBPCG W and P blocks: bands with skip_res[band] <=
  // skip_tol (soft-locked, so their columns are exactly zero) skip the FFT
  // passes and write zero output; null for every other transform
  const double* skip_res;
  double skip_tol;
};

}  // namespace ks

struct ks_plan {
  ks_grid grid;
  int32_t nb_max;
  int32_t prec;
  int64_t Ng;
  ks::Fft3 fft;
  void* tw[3];   // per-axis twiddles exp(-2 pi i t/n), plan precision
  int maxe_plane;  // elements per thread for the (y,z) plane passes
  int plane_threads; // threads per block of the plane passes (256 or 1024)
  int maxe_pencil; // elements per thread for the x-pencil pass
  int zc;          // z extent of one x-pencil tile
  size_t lds_plane;
  size_t lds_pencil;
  // Planes that do not fit in a CU's LDS (FP64 above 96^2 points): pass A and
  // pass C each run as two passes, z-transforms of groups of ry y-rows and
  // y-transforms of groups of zc2 z-columns of an x-plane.
  int split = 0;
  int ry = 0, zc2 = 0;
  size_t lds_rows = 0, lds_cols = 0;
  int a_parts = 0;  // partial sums per band written by the residual form of pass A
  // projectors, organised by blocks of kScatterPts consecutive grid points
  int32_t natoms = 0;
  int32_t nproj = 0;
  int32_t maxp = 0;             // max projectors per atom
  // Bloch vector != 0: every projector j of the caller's set is held as the
  // pair (2j, 2j + 1) of real projectors b cos(k.d), b sin(k.d), which the
  // reduction combines into the complex coefficient of b exp(-i k.d)
  int32_t kpairs = 0;
  int64_t nnz = 0;              // (point, projector) pairs with a support value
  int64_t nblk = 0;             // point blocks
  void* Dcoef = nullptr;        // nproj couplings, plan precision
  int32_t* blk_ptr = nullptr;   // nblk + 1: projectors blk_ptr[k].. touch block k
  int32_t* blk_proj = nullptr;  // global projector ids, ascending within a block
  int32_t maxl = 0;             // largest per-block projector count
  // scatter table, ELL by block: slot s of point t of block k at
  // (ell_ptr[k] + s) * kScatterPts + t holds (block-local projector, value);
  // unused slots hold (0, 0)
  int32_t* ell_ptr = nullptr;   // nblk + 1
  uint16_t* ell_lp = nullptr;
  void* ell_beta = nullptr;     // plan precision
  // projection table by boxes of grid points (tiles of tdim[0] x tdim[1] x
  // tdim[2], ntile[a] per axis, the last one per axis possibly partial):
  // tile k owns the (tile, atom) pairs tile_pair_ptr[k]..; pair q has the
  // entries pair_ent_ptr[q].. (tile-local points ascending, ent_t) and, from
  // pair_boff[q], the atom's np projector values at each of them (entry-major,
  // ent_beta); its partial coefficients are rows pair_row[q] .. + np of the
  // projection's partial buffer; projector p's rows, tiles ascending, are
  // proj_pairs[proj_pair_ptr[p]..]
  int32_t tdim[3] = {0, 0, 0};
  int32_t ntile[3] = {0, 0, 0};
  int64_t npairs = 0;
  int64_t nrows = 0;                 // partial rows (tile, projector)
  int32_t maxpt = 0;                 // most pairs in one tile
  int32_t budget = 0;                // projector values staged per batch
  int32_t* tile_pair_ptr = nullptr;  // ntiles + 1
  int32_t* pair_ent_ptr = nullptr;   // npairs + 1
  int32_t* pair_boff = nullptr;      // npairs + 1
  int32_t* pair_row = nullptr;       // npairs + 1
  uint16_t* ent_t = nullptr;
  void* ent_beta = nullptr;          // plan precision
  int32_t* proj_pair_ptr = nullptr;  // nproj + 1
  int32_t* proj_pairs = nullptr;     // nrows
};

namespace ks {

// ---- H-apply and preconditioner (fft.hip) ----
// With skip_res, bands whose skip_res[b] <= skip_tol have exactly zero
// columns (soft-locked W and P): their FFT passes are skipped and their
// output is written as zero.
template <typename T>
int apply_h(const ks_plan& p, const T* v, const c2<T>* psi, int64_t ldp, c2<T>* hpsi, int64_t ldh,
            int nb, c2<T>* tmp, c2<T>* dc, hipStream_t s, const double* skip_res = nullptr, double skip_tol = 0.0);

// E[b] = <x_b|T|x_b> for nb columns of X (uses tmp as scratch and
// `partial` of nb*n0*n1 doubles).
template <typename T>
int kinetic_energy(const ks_plan& p, const c2<T>* X, int64_t ld, int nb, c2<T>* tmp, double* partial,
                   double* E, hipStream_t s);

// R = AX - X theta -> res norms; W = precond(R) masked by res > lock_tol.
// partial: nb*n0 doubles; E: nb doubles (kinetic energies, TPA only).
template <typename T>
int precond_apply(const ks_plan& p, int kind, const c2<T>* X, const c2<T>* AX, const double* theta,
                  int64_t ld, int nb, double lock_tol, c2<T>* W, double* res, c2<T>* tmp,
                  double* partial, double* E, hipStream_t s);

size_t apply_h_work_bytes(const ks_plan& p, int nb);
// One real field through the periodic Poisson kernel 4 pi / |G|^2 (G = 0
// dropped): out = IFFT(4 pi / |G|^2 FFT(in)), complex buffers of Ng.
template <typename T>
int poisson(const ks_plan& p, const c2<T>* in, c2<T>* tmp, c2<T>* out, const double* one, hipStream_t s);
// Bytes of the nonlocal coefficient buffer of an H-apply (the coefficients
// and the per-tile partial sums of the projection).
size_t nl_dc_bytes(const ks_plan& p, int nb);
// Tile shape of the projection table for the plan's precision (each block
// stages tile x 16 bands of orbital values in LDS), and the kernel's LDS
// bytes for tiles of `tile_points` points, reals of `real_bytes`, at most
// maxpt pairs per tile and `budget` projector values staged at once.
void nl_tile_shape(int prec, const int n[3], int tdim[3]);
size_t nl_project_lds(int tile_points, size_t real_bytes, int maxpt, int budget);
size_t precond_work_bytes(const ks_plan& p, int nb);

// ---- the SCF loop's steps around the eigensolve (scf.hip) ----
size_t scf_work_bytes(const ks_plan& p);
int density_impl(const ks_plan& p, const void* X, int64_t ld, int nocc, const double* occ, double* n, hipStream_t s);
int hartree_impl(const ks_plan& p, const double* n, double* vh, void* work, hipStream_t s);
int lda_impl(const ks_plan& p, const double* n, double* vxc, double* exc, hipStream_t s);
int scf_potential_impl(const ks_plan& p, const double* n, const double* v_ion, void* v_eff, double* terms,
                       void* work, hipStream_t s);
int mix_impl(const ks_plan& p, double alpha, const double* n_in, const double* n_out, double* n_next, double* resid,
             void* work, hipStream_t s);

// ---- projected CG for training targets (cg.hip) ----
size_t jd_work_bytes(const ks_plan& p, int nb);
template <typename T>
int jd_correction(const ks_plan& p, const T* v, const c2<T>* X, const double* theta, const c2<T>* R, int64_t ld,
                  int nb, int maxit, double rtol, c2<T>* Tout, int32_t* iters, void* work, hipStream_t s);

// ---- learned preconditioner (cnn.hip) ----
constexpr int kCnnParams = 9106;
size_t cnn_act_floats(const ks_plan& p, int nbatch);
size_t cnn_backward_work(const ks_plan& p, int nbatch);
int cnn_forward_impl(const ks_plan& p, const float* params, int nbatch, const float* x, float* y, float* acts,
                     hipStream_t s);
int cnn_infer_impl(const ks_plan& p, const float* params, int nbatch, const float* x, float* y, float* buf,
                   hipStream_t s);
int cnn_backward_impl(const ks_plan& p, const float* params, int nbatch, const float* x, const float* acts,
                      const float* gy, float* grads, void* work, hipStream_t s);
int cnn_loss_impl(const float* y, const float* t, int nbatch, int64_t Ng, float* gy, double* loss, double* sums,
                  hipStream_t s);
int cnn_adam_impl(float* params, const float* grads, float* m, float* v, int n, int t, float lr, hipStream_t s);
int cnn_skip_impl(const ks_plan& p, int nbatch, const float* x, float* y, hipStream_t s);
int cnn_conv16_bf16_impl(const ks_plan& p, int nbatch, const float* x, const float* w, const float* b, bool silu,
                         float* y, hipStream_t s);
template <typename T>
int cnn_input_impl(const ks_plan& p, const c2<T>* R, int64_t ld, const double* rnorm, const T* V,
                   const double* theta, int nb, float* x, hipStream_t s);
template <typename T>
int cnn_output_impl(const ks_plan& p, const float* y, int nb, const double* res, double lock_tol, int32_t* bad,
                    c2<T>* W, int64_t ld,
                    hipStream_t s);

}  // namespace ks
