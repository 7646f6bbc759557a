// C ABI of the ksh library: plan construction, the H-apply and
// preconditioner entry points, the dense subspace solve, and the LOBPCG
// iteration that strings them together.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gemm.hpp"

namespace ks {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return KS_E_HIP - (int)e;
}

static inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

// ---------------------------------------------------------------- kernel timer
struct FamilyTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;  // begin/end pairs
  hipEvent_t open = nullptr;
};
static FamilyTimer g_timers[KS_KERNEL_FAMILIES];

void timer_begin(int f, hipStream_t s) {
  FamilyTimer& t = g_timers[f];
  if (!t.on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return;
  }
  t.open = e;
}

void timer_end(int f, hipStream_t s) {
  FamilyTimer& t = g_timers[f];
  if (!t.on || !t.open) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return;
  }
  t.ev.push_back(t.open);
  t.ev.push_back(e);
  t.open = nullptr;
}

// ---------------------------------------------------------------- plan helpers
static bool radix_plan(int n, AxisPlan& ap) {
  ap.n = n;
  ap.nst = 0;
  int m = n;
  // largest radices first: fewer LDS passes per transform
  const int order[8] = {16, 8, 7, 6, 5, 4, 3, 2};
  for (int r : order) {
    while (m % r == 0 && m > 1) {
      if (ap.nst >= kMaxStages) return false;
      ap.rad[ap.nst++] = r;
      m /= r;
    }
  }
  return m == 1 && n >= 1;
}

template <typename T>
static int upload_twiddles(int n, void** out) {
  std::vector<c2<T>> h(n);
  for (int t = 0; t < n; ++t) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)n;
    h[t].x = (T)cosl(ang);
    h[t].y = (T)sinl(ang);
  }
  KS_HIP(hipMalloc(out, sizeof(c2<T>) * std::max(n, 1)));
  KS_HIP(hipMemcpy(*out, h.data(), sizeof(c2<T>) * n, hipMemcpyHostToDevice));
  return 0;
}

template <typename T>
static int upload_vec(const std::vector<T>& h, T** out) {
  KS_HIP(hipMalloc(reinterpret_cast<void**>(out), sizeof(T) * std::max<size_t>(h.size(), 1)));
  if (!h.empty()) KS_HIP(hipMemcpy(*out, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return 0;
}

template <typename T>
static int upload_proj(ks_plan* p, const ks_projset* ps) {
  const int na = ps->n_atoms;
  const int32_t* sp = ps->atom_supp_ptr;
  const int32_t* si = ps->supp_idx;
  const int32_t* pp = ps->atom_proj_ptr;
  const int64_t* bp = ps->beta_ptr;
  std::vector<T> D(ps->n_proj);
  for (int i = 0; i < ps->n_proj; ++i) D[i] = (T)ps->D[i];
  // inverse table by grid point: entries (projector, value), projectors ascending
  std::vector<int32_t> cnt(p->Ng + 1, 0);
  for (int a = 0; a < na; ++a) {
    const int npa = pp[a + 1] - pp[a];
    for (int32_t s = sp[a]; s < sp[a + 1]; ++s) cnt[si[s] + 1] += npa;
  }
  for (int64_t r = 0; r < p->Ng; ++r) cnt[r + 1] += cnt[r];
  const int64_t nnz = cnt[p->Ng];
  if (nnz > INT32_MAX) return fail(KS_E_UNSUPPORTED, "projector table too large");
  std::vector<int32_t> pt_proj(nnz);
  std::vector<T> pt_beta(nnz);
  {
    std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int a = 0; a < na; ++a) {
      const int ns = sp[a + 1] - sp[a];
      for (int j = 0; j < pp[a + 1] - pp[a]; ++j) {
        for (int s = 0; s < ns; ++s) {
          const int r = si[sp[a] + s];
          const int32_t slot = fillp[r]++;
          pt_proj[slot] = pp[a] + j;
          pt_beta[slot] = (T)ps->beta[bp[a] + (int64_t)j * ns + s];
        }
      }
    }
  }
  // per block of kScatterPts points: the projectors its entries touch (its
  // rows), and the entries' projector ids rewritten as row-local indices
  const int64_t nblk = (p->Ng + kScatterPts - 1) / kScatterPts;
  std::vector<int32_t> blk_ptr(nblk + 1, 0), blk_proj;
  std::vector<int32_t> local(ps->n_proj, -1);
  int maxl = 0;
  for (int64_t k = 0; k < nblk; ++k) {
    const int64_t r0 = k * kScatterPts, r1 = std::min<int64_t>(p->Ng, r0 + kScatterPts);
    const size_t first = blk_proj.size();
    for (int32_t e = cnt[r0]; e < cnt[r1]; ++e)
      if (local[pt_proj[e]] < 0) {
        local[pt_proj[e]] = 0;
        blk_proj.push_back(pt_proj[e]);
      }
    std::sort(blk_proj.begin() + first, blk_proj.end());
    for (size_t i = first; i < blk_proj.size(); ++i) local[blk_proj[i]] = (int32_t)(i - first);
    for (int32_t e = cnt[r0]; e < cnt[r1]; ++e) pt_proj[e] = local[pt_proj[e]];
    for (size_t i = first; i < blk_proj.size(); ++i) local[blk_proj[i]] = -1;
    blk_ptr[k + 1] = (int32_t)blk_proj.size();
    maxl = std::max(maxl, (int)(blk_proj.size() - first));
  }
  if (maxl > 65535) return fail(KS_E_UNSUPPORTED, "too many projectors touch one block of grid points");
  // scatter: ELL slots per block
  std::vector<int32_t> ell_ptr(nblk + 1, 0);
  for (int64_t k = 0; k < nblk; ++k) {
    int wmax = 0;
    for (int64_t r = k * kScatterPts; r < std::min<int64_t>(p->Ng, (k + 1) * kScatterPts); ++r)
      wmax = std::max(wmax, cnt[r + 1] - cnt[r]);
    ell_ptr[k + 1] = ell_ptr[k] + wmax;
  }
  const int64_t nell = (int64_t)ell_ptr[nblk] * kScatterPts;
  std::vector<uint16_t> ell_lp(std::max<int64_t>(nell, 1), 0);
  std::vector<T> ell_beta(std::max<int64_t>(nell, 1), T(0));
  for (int64_t r = 0; r < p->Ng; ++r) {
    const int64_t k = r / kScatterPts, t = r - k * kScatterPts;
    for (int32_t e = cnt[r]; e < cnt[r + 1]; ++e) {
      const int64_t idx = ((int64_t)ell_ptr[k] + (e - cnt[r])) * kScatterPts + t;
      ell_lp[idx] = (uint16_t)pt_proj[e];
      ell_beta[idx] = pt_beta[e];
    }
  }
  if (blk_proj.empty()) blk_proj.push_back(0);
  p->natoms = na;
  p->nproj = ps->n_proj;
  p->nnz = nnz;
  p->nblk = nblk;
  p->maxl = maxl;
  int maxp = 0;
  for (int a = 0; a < na; ++a) maxp = std::max(maxp, pp[a + 1] - pp[a]);
  p->maxp = maxp;
  int rc;
  if ((rc = upload_vec(blk_ptr, &p->blk_ptr))) return rc;
  if ((rc = upload_vec(blk_proj, &p->blk_proj))) return rc;
  if ((rc = upload_vec(ell_ptr, &p->ell_ptr))) return rc;
  if ((rc = upload_vec(ell_lp, &p->ell_lp))) return rc;
  {
    std::vector<int32_t> spv(sp, sp + na + 1), siv(si, si + ps->n_supp), ppv(pp, pp + na + 1);
    std::vector<int64_t> bpv(bp, bp + na + 1);
    std::vector<T> bv(bp[na]);
    for (int64_t i = 0; i < bp[na]; ++i) bv[i] = (T)ps->beta[i];
    if ((rc = upload_vec(spv, &p->supp_ptr))) return rc;
    if ((rc = upload_vec(siv, &p->supp_idx))) return rc;
    if ((rc = upload_vec(ppv, &p->proj_ptr))) return rc;
    if ((rc = upload_vec(bpv, &p->beta_ptr))) return rc;
    T* b = nullptr;
    if ((rc = upload_vec(bv, &b))) return rc;
    p->beta = b;
  }
  T* d = nullptr;
  if ((rc = upload_vec(D, &d))) return rc;
  p->Dcoef = d;
  T* eb = nullptr;
  if ((rc = upload_vec(ell_beta, &eb))) return rc;
  p->ell_beta = eb;
  return 0;
}

// ---------------------------------------------------------------- small kernels
// d_i = active_i / sqrt(G_ii) (0 for a zero column), active_i = res_i > lock_tol
// when res is given.
__global__ void k_colscale(const double2* __restrict__ G, int ldg, int n, const double* __restrict__ res,
                           double lock_tol, double* __restrict__ dvec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double g = G[i + (int64_t)i * ldg].x;
  const bool act = res == nullptr || res[i] > lock_tol;
  dvec[i] = (act && g > 0.0) ? 1.0 / sqrt(g) : 0.0;
}

// G <- D G D, and a unit diagonal where d_i = 0.
__global__ void k_scale_gram(double2* __restrict__ G, int ldg, int n, const double* __restrict__ dvec) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    double2* g = G + i + (int64_t)j * ldg;
    const double s = dvec[i] * dvec[j];
    double2 v = make_double2(g->x * s, g->y * s);
    if (i == j && dvec[i] == 0.0) v = make_double2(1.0, 0.0);
    *g = v;
  }
}

__global__ void k_identity(double2* __restrict__ A, int lda, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    A[i + (int64_t)j * lda] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

// M = D Y (rows scaled) if the Cholesky succeeded, else M = D.  Written in the
// block precision.
template <typename T>
__global__ void k_cholqr_coef(const double2* __restrict__ Y, int ldy, int n, const double* __restrict__ dvec,
                              const int32_t* __restrict__ info, c2<T>* __restrict__ M, int ldm) {
  const int64_t total = (int64_t)n * n;
  const bool ok = *info == 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    double2 v;
    if (ok) {
      const double2 y = Y[i + (int64_t)j * ldy];
      v = make_double2(dvec[i] * y.x, dvec[i] * y.y);
    } else {
      v = make_double2(i == j ? dvec[i] : 0.0, 0.0);
    }
    M[i + (int64_t)j * ldm] = cmake<c2<T>>((T)v.x, (T)v.y);
  }
}

// Zero columns of the subspace basis: S_kk = 1, H_kk = 2 max|H_ii| + 1.
__global__ void k_decouple(double2* __restrict__ S, int lds, double2* __restrict__ H, int ldh, int m) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) mx = fmax(mx, fabs(H[i + (int64_t)i * ldh].x));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double big = 2.0 * mx + 1.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    if (S[i + (int64_t)i * lds].x == 0.0) {
      S[i + (int64_t)i * lds] = make_double2(1.0, 0.0);
      H[i + (int64_t)i * ldh] = make_double2(big, 0.0);
    }
  }
}

template <typename T>
__global__ void k_to_block(const double2* __restrict__ src, int ld_src, c2<T>* __restrict__ dst, int ld_dst, int rows,
                           int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows);
    const int64_t j = e / rows;
    const double2 v = src[i + j * ld_src];
    dst[i + j * ld_dst] = cmake<c2<T>>((T)v.x, (T)v.y);
  }
}

__global__ void k_copy_d(const double2* __restrict__ src, int ld_src, double2* __restrict__ dst, int ld_dst, int rows,
                         int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows);
    const int64_t j = e / rows;
    dst[i + j * ld_dst] = src[i + j * ld_src];
  }
}

static unsigned grid_for(int64_t total) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 4096)); }

// ---------------------------------------------------------------- workspace
struct LobWs {
  double2* S;   // m x m
  double2* H;
  double2* S0;
  double2* H0;
  double2* C;   // m x nb (FP64)
  void* Cb;     // m x nb block precision
  double2* G;   // nb x nb
  double2* Y;   // nb x nb
  void* M;      // nb x nb block precision
  double* dvec; // nb
  double* wnew; // m
  double* lam;  // nb, SVQB eigenvalues
  int32_t* info;  // 4 ints
  double* partial;
  double* E;
  void* dc;
  void* gram;
  void* hegv;
  void* potrf;
  double2* ttmp;
  int cnn_chunk;
  float* cnn_x;    // chunk x 3 x Ng
  float* cnn_buf;  // chunk x 32 x Ng
  float* cnn_y;    // chunk x 2 x Ng
  int32_t* cnn_bad; // chunk flags: non-finite network output
  double* cnn_norm;  // nb column norms of the TPA output
  double* cnn_part;  // column-norm partial sums of one chunk
  char* end;
};

static LobWs lob_ws(const ks_plan& p, void* work, int nb) {
  const int m = 3 * nb;
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  char* q = static_cast<char*>(work);
  LobWs w;
  auto take = [&](size_t bytes) { char* r = q; q += al(bytes); return r; };
  w.S = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.H = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.S0 = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.H0 = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.C = reinterpret_cast<double2*>(take((size_t)m * nb * 16));
  w.Cb = take((size_t)m * nb * es);
  w.G = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
  w.Y = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
  w.M = take((size_t)nb * nb * es);
  w.dvec = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.wnew = reinterpret_cast<double*>(take((size_t)m * 8));
  w.lam = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.info = reinterpret_cast<int32_t*>(take(16));
  const int n0 = p.fft.ax[0].n, n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  const size_t cnt = std::max<size_t>((size_t)n0, (size_t)n1 * (n2 / p.zc));
  w.partial = reinterpret_cast<double*>(take((size_t)nb * cnt * 8));
  w.E = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.dc = take((size_t)nb * std::max(p.nproj, 1) * es);
  w.gram = take(gram_work_bytes(m, p.Ng));
  w.hegv = take(hegv_work(m, nb));
  w.potrf = take(potrf_work(nb));
  w.ttmp = reinterpret_cast<double2*>(take((size_t)32 * std::max(nb, 1) * 16));
  w.cnn_chunk = std::min(nb, 32);
  w.cnn_x = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 3 * p.Ng * 4));
  w.cnn_buf = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 32 * p.Ng * 4));
  w.cnn_y = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 2 * p.Ng * 4));
  w.cnn_bad = reinterpret_cast<int32_t*>(take((size_t)w.cnn_chunk * 4));
  w.cnn_norm = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.cnn_part = reinterpret_cast<double*>(take(column_norms_partial(w.cnn_chunk) * 8));
  w.end = q;
  return w;
}

static size_t lobpcg_work_bytes(const ks_plan& p, int nb) {
  // lay the buffers out from a dummy aligned base and measure the span
  static char probe alignas(256);
  LobWs w = lob_ws(p, &probe, nb);
  return (size_t)(w.end - &probe);
}

// ---------------------------------------------------------------- LOBPCG pieces
template <typename T>
static BlockList<c2<T>> blist(const void* a, const void* b, const void* c, int64_t ld, int nb) {
  BlockList<c2<T>> L;
  L.p[0] = static_cast<const c2<T>*>(a);
  L.p[1] = static_cast<const c2<T>*>(b);
  L.p[2] = static_cast<const c2<T>*>(c);
  L.ld = ld;
  L.nb = nb;
  return L;
}

__global__ void k_zero_dead_diag(double2* __restrict__ G, int ldg, int n, const double* __restrict__ dvec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && dvec[i] == 0.0) G[i + (int64_t)i * ldg] = make_double2(0.0, 0.0);
}

static int read_info(const int32_t* dev, int32_t* host, hipStream_t s) {
  KS_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  KS_HIP(hipStreamSynchronize(s));
  return 0;
}

// SVQB coefficients: M[:, j] = d .* U[:, j] / sqrt(lam_j) when lam_j > tol *
// lam_max, else zero (lam ascending, so lam_max = lam[n-1]).
template <typename T>
__global__ void k_svqb_coef(const double2* __restrict__ U, int ldu, int n, const double* __restrict__ lam,
                            const double* __restrict__ dvec, double tol, c2<T>* __restrict__ M, int ldm) {
  const int64_t total = (int64_t)n * n;
  const double lmax = lam[n - 1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const bool keep = lam[j] > tol * lmax;
    const double sc = keep ? dvec[i] / sqrt(lam[j]) : 0.0;
    const double2 u = U[i + (int64_t)j * ldu];
    M[i + (int64_t)j * ldm] = cmake<c2<T>>((T)(sc * u.x), (T)(sc * u.y));
  }
}

// B <- B D L^-H (columns scaled to unit norm, then Cholesky-QR), written to
// out (and AB to aout when given).  If the Cholesky fails the block is
// orthonormalised through the eigenvectors of its scaled Gram matrix (SVQB)
// and directions with eigenvalue below svqb_tol * max become zero columns;
// this reads the Cholesky info back to the host.
template <typename T>
static int block_orthonormalise(const ks_plan& p, const LobWs& w, const void* B, const void* AB, void* out, void* aout,
                                int64_t ld, int nb, const double* res, double lock_tol, hipStream_t s) {
  int rc;
  auto L1 = blist<T>(B, nullptr, nullptr, ld, nb);
  if ((rc = gram<T>(L1, L1, nullptr, nb, p.Ng, w.G, nb, nullptr, 0, w.gram, s))) return rc;
  hipLaunchKernelGGL(k_colscale, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, w.G, nb, nb, res, lock_tol,
                     w.dvec);
  hipLaunchKernelGGL(k_scale_gram, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.G, nb, nb, w.dvec);
  KS_LAUNCH_CHECK("colscale");
  // keep the scaled Gram for the SVQB fallback, zero columns with a zero
  // diagonal so that they are dropped exactly
  hipLaunchKernelGGL(k_copy_d, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.G, nb, w.H0, nb, nb, nb);
  hipLaunchKernelGGL(k_zero_dead_diag, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, w.H0, nb, nb, w.dvec);
  if ((rc = potrf(nb, w.G, nb, w.potrf, w.info + 1, s))) return rc;
  int32_t hinfo = 0;
  if ((rc = read_info(w.info + 1, &hinfo, s))) return rc;
  if (hinfo == 0) {
    hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb);
    if ((rc = trsm('C', nb, nb, w.G, nb, w.Y, nb, w.potrf, w.ttmp, w.info + 1, s))) return rc;
    hipLaunchKernelGGL((k_cholqr_coef<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb, w.dvec,
                       w.info + 1, static_cast<c2<T>*>(w.M), nb);
    KS_LAUNCH_CHECK("cholqr_coef");
  } else {
    hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.S0, nb, nb);
    if ((rc = hegv(nb, nb, w.H0, nb, w.S0, nb, w.lam, w.C, nb, w.hegv, w.info + 2, s))) return rc;
    // S0 = I: only the tridiagonalisation's barrier can fail here
    if (nb >= hegv_resident_min_n()) {
      int32_t sinfo = 0;
      if ((rc = read_info(w.info + 2, &sinfo, s))) return rc;
      if (sinfo != 0) return fail(KS_E_NUMERIC, "SVQB eigensolve failed");
    }
    const double tol = p.prec == KS_FP64 ? 1e-12 : 1e-6;
    hipLaunchKernelGGL((k_svqb_coef<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.C, nb, nb, w.lam,
                       w.dvec, tol, static_cast<c2<T>*>(w.M), nb);
    KS_LAUNCH_CHECK("svqb_coef");
  }
  const auto* M = static_cast<const c2<T>*>(w.M);
  if ((rc = rotate<T>(L1, nb, nb, M, nb, nb, p.Ng, static_cast<c2<T>*>(out), nullptr, ld, s))) return rc;
  if (AB) {
    auto L2 = blist<T>(AB, nullptr, nullptr, ld, nb);
    if ((rc = rotate<T>(L2, nb, nb, M, nb, nb, p.Ng, static_cast<c2<T>*>(aout), nullptr, ld, s))) return rc;
  }
  return 0;
}

template <typename T>
static int lob_init(const ks_plan& p, const void* v, ks_lobpcg_state* st, void* work, hipStream_t s) {
  const int nb = st->nb;
  const int64_t ld = st->ld;
  LobWs w = lob_ws(p, work, nb);
  int rc;
  // Cholesky-QR of the start block
  auto LX = blist<T>(st->X, nullptr, nullptr, ld, nb);
  if ((rc = gram<T>(LX, LX, nullptr, nb, p.Ng, w.G, nb, nullptr, 0, w.gram, s))) return rc;
  if ((rc = potrf(nb, w.G, nb, w.potrf, w.info + 1, s))) return rc;
  int32_t hinfo = 0;
  if ((rc = read_info(w.info + 1, &hinfo, s))) return rc;
  if (hinfo != 0) return fail(KS_E_NUMERIC, "initial block is rank deficient");
  hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb);
  if ((rc = trsm('C', nb, nb, w.G, nb, w.Y, nb, w.potrf, w.ttmp, w.info + 1, s))) return rc;
  hipLaunchKernelGGL((k_to_block<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb,
                     static_cast<c2<T>*>(w.M), nb, nb, nb);
  KS_LAUNCH_CHECK("to_block");
  if ((rc = rotate<T>(LX, nb, nb, static_cast<const c2<T>*>(w.M), nb, nb, p.Ng, static_cast<c2<T>*>(st->Xn), nullptr,
                      ld, s)))
    return rc;
  std::swap(st->X, st->Xn);
  // AX = H X
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const c2<T>*>(st->X), ld,
                       static_cast<c2<T>*>(st->AX), ld, nb, static_cast<c2<T>*>(st->T1), static_cast<c2<T>*>(w.dc),
                       s)))
    return rc;
  // Rayleigh-Ritz on span(X)
  auto L1 = blist<T>(st->X, nullptr, nullptr, ld, nb);
  auto L2 = blist<T>(st->AX, nullptr, nullptr, ld, nb);
  if ((rc = gram<T>(L1, L1, &L2, nb, p.Ng, w.S, nb, w.H, nb, w.gram, s))) return rc;
  if ((rc = hegv(nb, nb, w.H, nb, w.S, nb, w.wnew, w.C, nb, w.hegv, w.info, s))) return rc;
  if ((rc = read_info(w.info, &hinfo, s))) return rc;
  if (hinfo != 0) return fail(KS_E_NUMERIC, "Rayleigh-Ritz of the initial block failed");
  hipLaunchKernelGGL((k_to_block<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.C, nb,
                     static_cast<c2<T>*>(w.Cb), nb, nb, nb);
  const auto* Cb = static_cast<const c2<T>*>(w.Cb);
  if ((rc = rotate<T>(L1, nb, nb, Cb, nb, nb, p.Ng, static_cast<c2<T>*>(st->Xn), nullptr, ld, s))) return rc;
  std::swap(st->X, st->Xn);
  // AX by a fresh H-apply of the rotated block (no rotation drift)
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const c2<T>*>(st->X), ld,
                       static_cast<c2<T>*>(st->AX), ld, nb, static_cast<c2<T>*>(st->T1), static_cast<c2<T>*>(w.dc),
                       s)))
    return rc;
  KS_HIP(hipMemcpyAsync(st->theta, w.wnew, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
  st->has_p = 0;
  st->iter = 0;
  st->last_info = 0;
  st->dropped_p = 0;
  return 0;
}

template <typename T>
static int lob_step(const ks_plan& p, const void* v, ks_lobpcg_state* st, const ks_lobpcg_opts* o, void* work,
                    hipStream_t s) {
  const int nb = st->nb;
  const int64_t ld = st->ld;
  LobWs w = lob_ws(p, work, nb);
  int rc;
  using T2 = c2<T>;
  // 1. residual, its norms, preconditioned and lock-masked W (into Xn)
  const bool learned = o->precond == KS_PRECOND_CNN || o->precond == KS_PRECOND_CNN_TPA;
  const int kind = o->precond == KS_PRECOND_CNN ? KS_PRECOND_NONE
                   : o->precond == KS_PRECOND_CNN_TPA ? KS_PRECOND_TPA
                                                      : o->precond;
  if ((rc = precond_apply<T>(p, kind, static_cast<const T2*>(st->X), static_cast<const T2*>(st->AX), st->theta, ld,
                             nb, o->lock_tol, static_cast<T2*>(st->Xn), st->res, static_cast<T2*>(st->T1), w.partial,
                             w.E, s)))
    return rc;
  if (learned) {
    // learned preconditioner, in band chunks, on the residual (CNN) or on
    // the TPA output with the skip connection (CNN_TPA)
    const bool skip = o->precond == KS_PRECOND_CNN_TPA;
    for (int b0 = 0; b0 < nb; b0 += w.cnn_chunk) {
      const int nc = std::min(w.cnn_chunk, nb - b0);
      T2* R = static_cast<T2*>(st->Xn) + (int64_t)b0 * ld;
      const double* nrm = st->res + b0;
      if (skip) {
        if ((rc = column_norms<T>(R, ld, nc, p.Ng, w.cnn_part, w.cnn_norm + b0, s))) return rc;
        nrm = w.cnn_norm + b0;
      }
      if ((rc = cnn_input_impl<T>(p, R, ld, nrm, static_cast<const T*>(v), st->theta + b0, nc, w.cnn_x, s)))
        return rc;
      if ((rc = cnn_infer_impl(p, o->cnn_params, nc, w.cnn_x, w.cnn_y, w.cnn_buf, s))) return rc;
      if (skip && (rc = cnn_skip_impl(p, nc, w.cnn_x, w.cnn_y, s))) return rc;
      if ((rc = cnn_output_impl<T>(p, w.cnn_y, nc, st->res + b0, o->lock_tol, w.cnn_bad, R, ld, s))) return rc;
    }
  }
  // 2. W <- W - X (X^H W), then W <- W D L^-H
  if ((rc = project_out<T>(static_cast<const T2*>(st->X), static_cast<const T2*>(st->Xn), static_cast<T2*>(st->W), ld,
                           nb, p.Ng, w.G, w.Cb, w.gram, s)))
    return rc;
  if ((rc = block_orthonormalise<T>(p, w, st->W, nullptr, st->Xn, nullptr, ld, nb, nullptr, 0.0, s))) return rc;
  std::swap(st->W, st->Xn);
  // 3. AW = H W
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->W), ld, static_cast<T2*>(st->AW), ld,
                       nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s)))
    return rc;
  // 4. P, AP masked and orthonormalised
  if (st->has_p) {
    if ((rc = block_orthonormalise<T>(p, w, st->P, nullptr, st->Pn, nullptr, ld, nb, st->res, o->lock_tol, s)))
      return rc;
    std::swap(st->P, st->Pn);
    if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->P), ld, static_cast<T2*>(st->AP), ld,
                         nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s)))
      return rc;
  }
  // 5. subspace matrices
  const int mfull = st->has_p ? 3 * nb : 2 * nb;
  auto LV = blist<T>(st->X, st->W, st->P, ld, nb);
  auto LAV = blist<T>(st->AX, st->AW, st->AP, ld, nb);
  if ((rc = gram<T>(LV, LV, &LAV, mfull, p.Ng, w.S, mfull, w.H, mfull, w.gram, s))) return rc;
  hipLaunchKernelGGL(k_decouple, dim3(1), dim3(256), 0, s, w.S, mfull, w.H, mfull, mfull);
  KS_LAUNCH_CHECK("decouple");
  if (st->has_p) {
    hipLaunchKernelGGL(k_copy_d, dim3(grid_for((int64_t)mfull * mfull)), dim3(256), 0, s, w.S, mfull, w.S0, mfull,
                       mfull, mfull);
    hipLaunchKernelGGL(k_copy_d, dim3(grid_for((int64_t)mfull * mfull)), dim3(256), 0, s, w.H, mfull, w.H0, mfull,
                       mfull, mfull);
  }
  // 6. reduction and eigensolve; drop P on a failed Cholesky
  int m = mfull;
  if ((rc = hegv(m, nb, w.H, mfull, w.S, mfull, w.wnew, w.C, m, w.hegv, w.info, s))) return rc;
  int32_t hinfo = 0;
  if ((rc = read_info(w.info, &hinfo, s))) return rc;
  if (hinfo < 0) return fail(KS_E_NUMERIC, "subspace eigensolve: tridiagonalisation grid barrier timed out");
  if (hinfo != 0 && st->has_p) {
    st->dropped_p += 1;
    m = 2 * nb;
    hipLaunchKernelGGL(k_copy_d, dim3(grid_for((int64_t)mfull * mfull)), dim3(256), 0, s, w.S0, mfull, w.S, mfull,
                       mfull, mfull);
    hipLaunchKernelGGL(k_copy_d, dim3(grid_for((int64_t)mfull * mfull)), dim3(256), 0, s, w.H0, mfull, w.H, mfull,
                       mfull, mfull);
    if ((rc = hegv(m, nb, w.H, mfull, w.S, mfull, w.wnew, w.C, m, w.hegv, w.info, s))) return rc;
    if ((rc = read_info(w.info, &hinfo, s))) return rc;
    if (hinfo < 0) return fail(KS_E_NUMERIC, "subspace eigensolve: tridiagonalisation grid barrier timed out");
  }
  st->last_info = hinfo;
  if (hinfo != 0) return fail(KS_E_NUMERIC, "subspace overlap is not positive definite");
  // 7. rotation: X <- V C and P <- V[:, nb:] C[nb:, :] in one pass over V
  hipLaunchKernelGGL((k_to_block<T>), dim3(grid_for((int64_t)m * nb)), dim3(256), 0, s, w.C, m,
                     static_cast<T2*>(w.Cb), m, m, nb);
  KS_LAUNCH_CHECK("to_block");
  const auto* Cb = static_cast<const T2*>(w.Cb);
  if ((rc = rotate<T>(LV, m, nb, Cb, m, nb, p.Ng, static_cast<T2*>(st->Xn), static_cast<T2*>(st->Pn), ld, s)))
    return rc;
  std::swap(st->X, st->Xn);
  std::swap(st->P, st->Pn);
  // 8. mixed plans: FP64-factor Cholesky-QR of X
  if (p.prec != KS_FP64) {
    if ((rc = block_orthonormalise<T>(p, w, st->X, nullptr, st->Xn, nullptr, ld, nb, nullptr, 0.0, s))) return rc;
    std::swap(st->X, st->Xn);
  }
  // 9. AX by a fresh H-apply (AP is formed the same way next step)
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->X), ld, static_cast<T2*>(st->AX), ld,
                       nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s)))
    return rc;
  KS_HIP(hipMemcpyAsync(st->theta, w.wnew, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
  st->has_p = 1;
  st->iter += 1;
  return 0;
}

}  // namespace ks

using namespace ks;

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* ks_last_error(void) { return g_last_error.c_str(); }

int ks_kernel_timer(int32_t enable, int32_t family) {
  if (family < 0 || family >= KS_KERNEL_FAMILIES) return fail(-2, "unknown kernel family");
  FamilyTimer& t = g_timers[family];
  if (enable) {
    for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
    t.ev.clear();
  }
  t.on = enable != 0;
  return 0;
}

int ks_kernel_timer_read(int32_t family, double* total_ms, int64_t* launches) {
  if (family < 0 || family >= KS_KERNEL_FAMILIES) return fail(-1, "unknown kernel family");
  if (!total_ms) return fail(-2, "total_ms is null");
  if (!launches) return fail(-3, "launches is null");
  FamilyTimer& t = g_timers[family];
  double sum = 0.0;
  for (size_t i = 0; i + 1 < t.ev.size(); i += 2) {
    KS_HIP(hipEventSynchronize(t.ev[i + 1]));
    float ms = 0.f;
    KS_HIP(hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]));
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)(t.ev.size() / 2);
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t.ev.clear();
  return 0;
}

int ks_plan_create(ks_plan** out, const ks_grid* grid, const ks_projset* proj, int32_t nb_max, int32_t precision,
                   void* stream) {
  g_last_error.clear();
  if (!out) return fail(-1, "out is null");
  if (!grid) return fail(-2, "grid is null");
  if (nb_max <= 0) return fail(-4, "nb_max must be positive");
  if (3 * (int64_t)nb_max > kHegvMaxN) return fail(-4, "nb_max too large: the subspace problem of order 3 nb_max must be at most 3700");
  if (precision < KS_FP64 || precision > KS_MIXED_BF16X3) return fail(-5, "unknown precision");
  if (precision == KS_MIXED_BF16X3) return fail(KS_E_UNSUPPORTED, "the bf16x3 Gram split is not built");
  ks_plan* p = new ks_plan();
  p->grid = *grid;
  p->nb_max = nb_max;
  p->prec = precision;
  p->Ng = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1 || !(grid->L[a] > 0.0) || !radix_plan(grid->n[a], p->fft.ax[a])) {
      delete p;
      return fail(-2, "grid sizes must be positive products of 2, 3, 5, 7 and L positive");
    }
    p->fft.twopi_over_L[a] = 2.0 * M_PI / grid->L[a];
    p->Ng *= grid->n[a];
  }
  const size_t es = precision == KS_FP64 ? 16 : 8;
  const int n0 = grid->n[0], n1 = grid->n[1], n2 = grid->n[2];
  const int plane = n1 * n2;
  // planes above 4096 points use 1024-thread blocks: one or two such planes
  // fill a CU's LDS, and the larger block keeps 16 or more waves resident
  p->plane_threads = (plane > 4096 && plane <= 16384) ? 1024 : kThreads;
  const int ept = (int)ceil_div(plane, p->plane_threads);
  const int choices[5] = {4, 12, 16, 48, 64};
  p->maxe_plane = 0;
  for (int c : choices)
    if (ept <= c && (c != 12 || p->plane_threads == 1024)) { p->maxe_plane = c; break; }
  if (p->maxe_plane == 0) { delete p; return fail(KS_E_UNSUPPORTED, "plane too large"); }
  p->zc = 1;
  for (int z = 1; z <= n2; ++z)
    if (n2 % z == 0 && (int64_t)n0 * z <= 16 * kThreads) p->zc = z;
  p->maxe_pencil = 16;
  if ((int64_t)n0 > 16 * kThreads) { delete p; return fail(KS_E_UNSUPPORTED, "x extent too large"); }
  // data (planes padded: one pad element per 16) plus the staged twiddle tables
  p->lds_plane = (size_t)(plane + (plane >> 4) + 1 + n1 + n2) * es;
  p->lds_pencil = (size_t)(n0 * p->zc + n0) * es;
  int dev = 0, maxlds = 0;
  KS_HIP(hipGetDevice(&dev));
  KS_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (p->lds_plane > (size_t)maxlds || p->lds_pencil > (size_t)maxlds) {
    delete p;
    return fail(KS_E_UNSUPPORTED, "plane does not fit in LDS");
  }
  int rc = 0;
  for (int a = 0; a < 3 && rc == 0; ++a)
    rc = precision == KS_FP64 ? upload_twiddles<double>(grid->n[a], &p->tw[a]) : upload_twiddles<float>(grid->n[a], &p->tw[a]);
  if (rc == 0 && proj && proj->n_proj > 0) {
    if (!proj->atom_supp_ptr || !proj->supp_idx || !proj->atom_proj_ptr || !proj->beta_ptr || !proj->beta || !proj->D) {
      ks_plan_destroy(p);
      return fail(-3, "projector set has null arrays");
    }
    for (int64_t i = 0; i < proj->n_supp; ++i)
      if (proj->supp_idx[i] < 0 || proj->supp_idx[i] >= p->Ng) {
        ks_plan_destroy(p);
        return fail(-3, "support index out of the grid");
      }
    if (proj->atom_proj_ptr[proj->n_atoms] != proj->n_proj || proj->atom_supp_ptr[proj->n_atoms] != proj->n_supp) {
      ks_plan_destroy(p);
      return fail(-3, "projector CSR pointers inconsistent");
    }
    rc = precision == KS_FP64 ? upload_proj<double>(p, proj) : upload_proj<float>(p, proj);
  }
  if (rc) {
    ks_plan_destroy(p);
    return rc;
  }
  KS_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  *out = p;
  return 0;
}

int ks_plan_destroy(ks_plan* p) {
  if (!p) return 0;
  for (int a = 0; a < 3; ++a) (void)hipFree(p->tw[a]);
  void* bufs[] = {p->Dcoef,   p->blk_ptr,  p->blk_proj, p->ell_ptr,  p->ell_lp, p->ell_beta,
                  p->supp_ptr, p->supp_idx, p->proj_ptr, p->beta_ptr, p->beta};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
  return 0;
}

int ks_workspace_size(const ks_plan* p, int32_t op, int32_t nb, size_t* bytes) {
  if (!p) return fail(-1, "plan is null");
  if (nb <= 0 || nb > p->nb_max) return fail(-3, "nb out of range");
  if (!bytes) return fail(-4, "bytes is null");
  switch (op) {
    case KS_OP_APPLY_H: *bytes = apply_h_work_bytes(*p, nb); return 0;
    case KS_OP_PRECOND: *bytes = precond_work_bytes(*p, nb); return 0;
    case KS_OP_LOBPCG: *bytes = lobpcg_work_bytes(*p, nb); return 0;
    case KS_OP_JD: *bytes = jd_work_bytes(*p, nb); return 0;
    default: return fail(-2, "unknown op");
  }
}

int ks_apply_h(const ks_plan* p, const void* v_loc, const void* psi, int64_t ld_psi, void* hpsi, int64_t ld_hpsi,
               int32_t nb, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!v_loc) return fail(-2, "v_loc is null");
  if (!psi) return fail(-3, "psi is null");
  if (ld_psi < p->Ng) return fail(-4, "ld_psi < Ng");
  if (!hpsi) return fail(-5, "hpsi is null");
  if (ld_hpsi < p->Ng) return fail(-6, "ld_hpsi < Ng");
  if (nb <= 0 || nb > p->nb_max) return fail(-7, "nb out of range");
  if (!work) return fail(-8, "work is null");
  const size_t need = apply_h_work_bytes(*p, nb);
  if (work_bytes < need) return fail(KS_E_WORKSPACE, "workspace too small");
  const size_t es = p->prec == KS_FP64 ? 16 : 8;
  char* tmp = static_cast<char*>(work);
  char* dc = tmp + al((size_t)p->Ng * nb * es);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return apply_h<double>(*p, static_cast<const double*>(v_loc), static_cast<const double2*>(psi), ld_psi,
                           static_cast<double2*>(hpsi), ld_hpsi, nb, reinterpret_cast<double2*>(tmp),
                           reinterpret_cast<double2*>(dc), s);
  return apply_h<float>(*p, static_cast<const float*>(v_loc), static_cast<const float2*>(psi), ld_psi,
                        static_cast<float2*>(hpsi), ld_hpsi, nb, reinterpret_cast<float2*>(tmp),
                        reinterpret_cast<float2*>(dc), s);
}

int ks_precond_apply(const ks_plan* p, int32_t kind, const void* X, const void* AX, const double* theta, int64_t ld,
                     int32_t nb, double lock_tol, void* W, double* res, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (kind != KS_PRECOND_NONE && kind != KS_PRECOND_TPA) return fail(-2, "unknown preconditioner");
  if (!X) return fail(-3, "X is null");
  if (!AX) return fail(-4, "AX is null");
  if (!theta) return fail(-5, "theta is null");
  if (ld < p->Ng) return fail(-6, "ld < Ng");
  if (nb <= 0 || nb > p->nb_max) return fail(-7, "nb out of range");
  if (!W) return fail(-9, "W is null");
  if (!res) return fail(-10, "res is null");
  if (!work) return fail(-11, "work is null");
  if (work_bytes < precond_work_bytes(*p, nb)) return fail(KS_E_WORKSPACE, "workspace too small");
  const size_t es = p->prec == KS_FP64 ? 16 : 8;
  char* tmp = static_cast<char*>(work);
  const int n0 = p->fft.ax[0].n, n1 = p->fft.ax[1].n, n2 = p->fft.ax[2].n;
  const size_t cnt = std::max<size_t>((size_t)n0, (size_t)n1 * (n2 / p->zc));
  double* partial = reinterpret_cast<double*>(tmp + al((size_t)p->Ng * nb * es));
  double* E = reinterpret_cast<double*>(reinterpret_cast<char*>(partial) + al((size_t)nb * cnt * 8));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return precond_apply<double>(*p, kind, static_cast<const double2*>(X), static_cast<const double2*>(AX), theta, ld,
                                 nb, lock_tol, static_cast<double2*>(W), res, reinterpret_cast<double2*>(tmp), partial,
                                 E, s);
  return precond_apply<float>(*p, kind, static_cast<const float2*>(X), static_cast<const float2*>(AX), theta, ld, nb,
                              lock_tol, static_cast<float2*>(W), res, reinterpret_cast<float2*>(tmp), partial, E, s);
}

int hegv_workspace_size(int32_t n, int32_t nev, size_t* bytes) {
  if (n <= 0 || n > kHegvMaxN) return fail(-1, "n out of range (1..3700: the inverse iteration stages 44 bytes per row in LDS)");
  if (nev <= 0 || nev > n) return fail(-2, "nev out of range");
  if (!bytes) return fail(-3, "bytes is null");
  *bytes = hegv_work(n, nev);
  return 0;
}

int hegv_reduce_solve(int32_t n, int32_t nev, void* H, int32_t ldh, void* S, int32_t lds, double* w, void* C,
                      int32_t ldc, void* work, size_t work_bytes, int32_t* info_dev, void* stream) {
  g_last_error.clear();
  if (n <= 0 || n > kHegvMaxN) return fail(-1, "n out of range (1..3700: the inverse iteration stages 44 bytes per row in LDS)");
  if (nev <= 0 || nev > n) return fail(-2, "nev out of range");
  if (!H) return fail(-3, "H is null");
  if (ldh < n) return fail(-4, "ldh < n");
  if (!S) return fail(-5, "S is null");
  if (lds < n) return fail(-6, "lds < n");
  if (!w) return fail(-7, "w is null");
  if (!C) return fail(-8, "C is null");
  if (ldc < n) return fail(-9, "ldc < n");
  if (!work) return fail(-10, "work is null");
  if (work_bytes < hegv_work(n, nev)) return fail(KS_E_WORKSPACE, "workspace too small");
  if (!info_dev) return fail(-12, "info is null");
  return hegv(n, nev, static_cast<double2*>(H), ldh, static_cast<double2*>(S), lds, w, static_cast<double2*>(C), ldc,
              work, info_dev, static_cast<hipStream_t>(stream));
}

static int check_state(const ks_plan* p, const ks_lobpcg_state* st) {
  if (!p) return fail(-1, "plan is null");
  if (!st) return fail(-3, "state is null");
  if (st->nb <= 0 || st->nb > p->nb_max) return fail(-3, "state nb out of range");
  if (st->ld < p->Ng) return fail(-3, "state ld < Ng");
  const void* ptrs[] = {st->X, st->AX, st->W, st->AW, st->P, st->AP, st->Xn, st->AXn, st->Pn, st->APn, st->T1,
                        st->theta, st->res};
  for (const void* q : ptrs)
    if (!q) return fail(-3, "state has a null buffer");
  return 0;
}

int lobpcg_init(const ks_plan* p, const void* v_loc, ks_lobpcg_state* st, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  int rc = check_state(p, st);
  if (rc) return rc;
  if (!v_loc) return fail(-2, "v_loc is null");
  if (!work) return fail(-4, "work is null");
  if (work_bytes < lobpcg_work_bytes(*p, st->nb)) return fail(KS_E_WORKSPACE, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->prec == KS_FP64 ? lob_init<double>(*p, v_loc, st, work, s) : lob_init<float>(*p, v_loc, st, work, s);
}

int lobpcg_step(const ks_plan* p, const void* v_loc, ks_lobpcg_state* st, const ks_lobpcg_opts* opts, void* work,
                size_t work_bytes, void* stream) {
  g_last_error.clear();
  int rc = check_state(p, st);
  if (rc) return rc;
  if (!v_loc) return fail(-2, "v_loc is null");
  if (!opts) return fail(-4, "opts is null");
  if (opts->precond != KS_PRECOND_NONE && opts->precond != KS_PRECOND_TPA && opts->precond != KS_PRECOND_CNN &&
      opts->precond != KS_PRECOND_CNN_TPA)
    return fail(-4, "unknown preconditioner");
  if ((opts->precond == KS_PRECOND_CNN || opts->precond == KS_PRECOND_CNN_TPA) && !opts->cnn_params)
    return fail(-4, "CNN preconditioner without parameters");
  if (!work) return fail(-5, "work is null");
  if (work_bytes < lobpcg_work_bytes(*p, st->nb)) return fail(KS_E_WORKSPACE, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->prec == KS_FP64 ? lob_step<double>(*p, v_loc, st, opts, work, s)
                            : lob_step<float>(*p, v_loc, st, opts, work, s);
}

}  // extern "C"

// ---------------------------------------------------------------- learned preconditioner ABI
extern "C" {

int ks_jd_correction(const ks_plan* p, const void* v_loc, const void* X, const double* theta, const void* R, int64_t ld,
                     int32_t nb, int32_t maxit, double rtol, void* Tout, int32_t* iters, void* work, size_t work_bytes,
                     void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!v_loc) return fail(-2, "v_loc is null");
  if (!X) return fail(-3, "X is null");
  if (!theta) return fail(-4, "theta is null");
  if (!R) return fail(-5, "R is null");
  if (ld < p->Ng) return fail(-6, "ld < Ng");
  if (nb <= 0 || nb > p->nb_max) return fail(-7, "nb out of range");
  if (maxit < 0) return fail(-8, "maxit negative");
  if (!(rtol >= 0.0)) return fail(-9, "rtol negative");
  if (!Tout) return fail(-10, "T is null");
  if (!iters) return fail(-11, "iters is null");
  if (!work) return fail(-12, "work is null");
  if (work_bytes < jd_work_bytes(*p, nb)) return fail(KS_E_WORKSPACE, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return jd_correction<double>(*p, static_cast<const double*>(v_loc), static_cast<const double2*>(X), theta,
                                 static_cast<const double2*>(R), ld, nb, maxit, rtol, static_cast<double2*>(Tout), iters,
                                 work, s);
  return jd_correction<float>(*p, static_cast<const float*>(v_loc), static_cast<const float2*>(X), theta,
                              static_cast<const float2*>(R), ld, nb, maxit, rtol, static_cast<float2*>(Tout), iters,
                              work, s);
}

int cnn_workspace_size(const ks_plan* p, int32_t nbatch, size_t* act_floats, size_t* work_bytes) {
  if (!p) return fail(-1, "plan is null");
  if (nbatch <= 0) return fail(-2, "nbatch must be positive");
  if (!act_floats) return fail(-3, "act_floats is null");
  if (!work_bytes) return fail(-4, "work_bytes is null");
  *act_floats = cnn_act_floats(*p, nbatch);
  *work_bytes = cnn_backward_work(*p, nbatch);
  return 0;
}

int cnn_forward(const ks_plan* p, const float* params, int32_t nbatch, const float* x, float* y, float* acts,
                void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!params) return fail(-2, "params is null");
  if (nbatch <= 0) return fail(-3, "nbatch must be positive");
  if (!x) return fail(-4, "x is null");
  if (!y) return fail(-5, "y is null");
  if (!acts) return fail(-6, "acts is null");
  return cnn_forward_impl(*p, params, nbatch, x, y, acts, static_cast<hipStream_t>(stream));
}

int cnn_backward(const ks_plan* p, const float* params, int32_t nbatch, const float* x, const float* acts,
                 const float* gy, float* grads, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!params) return fail(-2, "params is null");
  if (nbatch <= 0) return fail(-3, "nbatch must be positive");
  if (!x) return fail(-4, "x is null");
  if (!acts) return fail(-5, "acts is null");
  if (!gy) return fail(-6, "gy is null");
  if (!grads) return fail(-7, "grads is null");
  if (!work) return fail(-8, "work is null");
  if (work_bytes < cnn_backward_work(*p, nbatch)) return fail(KS_E_WORKSPACE, "workspace too small");
  return cnn_backward_impl(*p, params, nbatch, x, acts, gy, grads, work, static_cast<hipStream_t>(stream));
}

int cnn_loss(int32_t nbatch, int64_t Ng, const float* y, const float* t, float* gy, double* loss, double* sums,
             void* stream) {
  g_last_error.clear();
  if (nbatch <= 0) return fail(-1, "nbatch must be positive");
  if (Ng <= 0) return fail(-2, "Ng must be positive");
  if (!y) return fail(-3, "y is null");
  if (!t) return fail(-4, "t is null");
  if (!gy) return fail(-5, "gy is null");
  if (!loss) return fail(-6, "loss is null");
  if (!sums) return fail(-7, "sums is null");
  return cnn_loss_impl(y, t, nbatch, Ng, gy, loss, sums, static_cast<hipStream_t>(stream));
}

int cnn_adam_step(float* params, const float* grads, float* m, float* v, int32_t nparam, int32_t t, float lr,
                  void* stream) {
  g_last_error.clear();
  if (!params) return fail(-1, "params is null");
  if (!grads) return fail(-2, "grads is null");
  if (!m) return fail(-3, "m is null");
  if (!v) return fail(-4, "v is null");
  if (nparam <= 0) return fail(-5, "nparam must be positive");
  if (t < 1) return fail(-6, "t counts from 1");
  return cnn_adam_impl(params, grads, m, v, nparam, t, lr, static_cast<hipStream_t>(stream));
}

int cnn_make_input(const ks_plan* p, const void* R, int64_t ld, const double* rnorm, const void* v_loc,
                   const double* theta, int32_t nb, float* x, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!R) return fail(-2, "R is null");
  if (ld < p->Ng) return fail(-3, "ld < Ng");
  if (!v_loc) return fail(-5, "v_loc is null");
  if (!theta) return fail(-6, "theta is null");
  if (nb <= 0) return fail(-7, "nb must be positive");
  if (!x) return fail(-8, "x is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return cnn_input_impl<double>(*p, static_cast<const double2*>(R), ld, rnorm, static_cast<const double*>(v_loc),
                                  theta, nb, x, s);
  return cnn_input_impl<float>(*p, static_cast<const float2*>(R), ld, rnorm, static_cast<const float*>(v_loc), theta,
                               nb, x, s);
}

int cnn_infer(const ks_plan* p, const float* params, int32_t nbatch, const float* x, float* y, float* buf,
              void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!params) return fail(-2, "params is null");
  if (nbatch <= 0) return fail(-3, "nbatch must be positive");
  if (!x) return fail(-4, "x is null");
  if (!y) return fail(-5, "y is null");
  if (!buf) return fail(-6, "buf is null");
  return cnn_infer_impl(*p, params, nbatch, x, y, buf, static_cast<hipStream_t>(stream));
}

int cnn_conv16_bf16(const ks_plan* p, int32_t nbatch, const float* x, const float* w, const float* b, int32_t silu,
                    float* y, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (nbatch <= 0) return fail(-2, "nbatch must be positive");
  if (!x) return fail(-3, "x is null");
  if (!w) return fail(-4, "w is null");
  if (!b) return fail(-5, "b is null");
  if (!y) return fail(-7, "y is null");
  if (x == y) return fail(-7, "y must not alias x");
  return cnn_conv16_bf16_impl(*p, nbatch, x, w, b, silu != 0, y, static_cast<hipStream_t>(stream));
}

int cnn_add_skip(const ks_plan* p, int32_t nbatch, const float* x, float* y, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (nbatch <= 0) return fail(-2, "nbatch must be positive");
  if (!x) return fail(-3, "x is null");
  if (!y) return fail(-4, "y is null");
  return cnn_skip_impl(*p, nbatch, x, y, static_cast<hipStream_t>(stream));
}

}  // extern "C"
