// C ABI of the ksh library: plan construction, the H-apply and
// preconditioner entry points, the dense subspace solve, and the LOBPCG
// iteration that strings them together.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
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
// set while an entry point that must not create runtime objects runs
static thread_local bool g_timers_suppressed = false;

void timer_begin(int f, hipStream_t s) {
  FamilyTimer& t = g_timers[f];
  if (!t.on || g_timers_suppressed) return;
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
  if (!t.on || !t.open || g_timers_suppressed) return;
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

// Largest work item of the tiled projection (entries of one atom in one
// tile): items of up to 96 entries give the 16 waves of a block even shares
// (whole (tile, atom) pairs left three of them idle and the busiest with
// 2.3 times the mean on the 216-atom cell), at the price of more partial
// rows to reduce.
constexpr int kPairChunk = 96;

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
  // projection table by tiles of grid points: (tile, atom) pairs, tiles in
  // order and atoms ascending within a tile; a pair's entries are the atom's
  // support points inside the tile (ascending) with its np projector values
  {
    const int n[3] = {p->fft.ax[0].n, p->fft.ax[1].n, p->fft.ax[2].n};
    nl_tile_shape(p->prec, n, p->tdim);
    for (int a2 = 0; a2 < 3; ++a2) p->ntile[a2] = (int32_t)ceil_div(n[a2], p->tdim[a2]);
    const int64_t ntiles = (int64_t)p->ntile[0] * p->ntile[1] * p->ntile[2];
    // (tile, atom, support index) triples, bucketed by tile in atom order
    std::vector<int32_t> tcount(ntiles + 1, 0);
    std::vector<int64_t> tile_of(ps->n_supp);
    std::vector<uint16_t> local_of(ps->n_supp);
    for (int a = 0; a < na; ++a) {
      if (pp[a + 1] == pp[a]) continue;
      for (int32_t s2 = sp[a]; s2 < sp[a + 1]; ++s2) {
        const int64_t r = si[s2];
        const int z = (int)(r % n[2]), y = (int)((r / n[2]) % n[1]), x = (int)(r / ((int64_t)n[1] * n[2]));
        tile_of[s2] = ((int64_t)(x / p->tdim[0]) * p->ntile[1] + y / p->tdim[1]) * p->ntile[2] + z / p->tdim[2];
        local_of[s2] = (uint16_t)(((x % p->tdim[0]) * p->tdim[1] + y % p->tdim[1]) * p->tdim[2] + z % p->tdim[2]);
        tcount[tile_of[s2] + 1] += 1;
      }
    }
    for (int64_t k = 0; k < ntiles; ++k) tcount[k + 1] += tcount[k];
    std::vector<int32_t> slot(tcount[ntiles]);  // support indices grouped by tile, atoms ascending
    {
      std::vector<int32_t> fill(tcount.begin(), tcount.end() - 1);
      for (int a = 0; a < na; ++a) {
        if (pp[a + 1] == pp[a]) continue;
        for (int32_t s2 = sp[a]; s2 < sp[a + 1]; ++s2) slot[fill[tile_of[s2]]++] = s2;
      }
    }
    std::vector<int32_t> atom_of_supp(ps->n_supp);
    for (int a = 0; a < na; ++a)
      for (int32_t s2 = sp[a]; s2 < sp[a + 1]; ++s2) atom_of_supp[s2] = a;
    std::vector<int32_t> tile_pair_ptr(ntiles + 1, 0), pair_ent_ptr(1, 0), pair_boff(1, 0), pair_row(1, 0),
        pair_atom;
    std::vector<uint16_t> ent_t;
    std::vector<T> ent_beta;
    ent_t.reserve(tcount[ntiles]);
    ent_beta.reserve(nnz);
    for (int64_t k = 0; k < ntiles; ++k) {
      for (int32_t i = tcount[k]; i < tcount[k + 1];) {
        const int a = atom_of_supp[slot[i]];
        const int npa = pp[a + 1] - pp[a];
        const int ns = sp[a + 1] - sp[a];
        int32_t j = i;
        // the atom's support is ascending in grid index; within a tile the
        // local index is then ascending too only per z-run, so sort
        std::vector<std::pair<uint16_t, int32_t>> pts;
        for (; j < tcount[k + 1] && atom_of_supp[slot[j]] == a; ++j) pts.push_back({local_of[slot[j]], slot[j]});
        std::sort(pts.begin(), pts.end());
        // a pair is one wave's work item: an atom covering much of the tile
        // is cut into items of at most kPairChunk entries (each with its
        // own partial rows, reduced in order with the rest), so that the
        // waves of a block get even shares
        for (size_t c0 = 0; c0 < pts.size(); c0 += kPairChunk) {
          const size_t c1 = std::min(pts.size(), c0 + (size_t)kPairChunk);
          for (size_t e = c0; e < c1; ++e) {
            ent_t.push_back(pts[e].first);
            const int32_t s2 = pts[e].second - sp[a];
            for (int jp = 0; jp < npa; ++jp) ent_beta.push_back((T)ps->beta[bp[a] + (int64_t)jp * ns + s2]);
          }
          pair_atom.push_back(a);
          pair_ent_ptr.push_back((int32_t)ent_t.size());
          pair_boff.push_back((int32_t)ent_beta.size());
          pair_row.push_back(pair_row.back() + npa);
        }
        i = j;
      }
      tile_pair_ptr[k + 1] = (int32_t)pair_atom.size();
    }
    const int64_t npairs = (int64_t)pair_atom.size();
    const int64_t nrows = pair_row.back();
    if ((int64_t)ent_beta.size() > INT32_MAX || nrows > INT32_MAX)
      return fail(KS_E_UNSUPPORTED, "projector table too large");
    // projector -> its partial rows, tiles ascending
    std::vector<int32_t> proj_pair_ptr(ps->n_proj + 1, 0), proj_pairs(std::max<int64_t>(nrows, 1));
    for (int64_t q = 0; q < npairs; ++q)
      for (int jp = pp[pair_atom[q]]; jp < pp[pair_atom[q] + 1]; ++jp) proj_pair_ptr[jp + 1] += 1;
    for (int i = 0; i < ps->n_proj; ++i) proj_pair_ptr[i + 1] += proj_pair_ptr[i];
    {
      std::vector<int32_t> fill(proj_pair_ptr.begin(), proj_pair_ptr.end() - 1);
      for (int64_t q = 0; q < npairs; ++q) {
        const int a = pair_atom[q];
        for (int jp = 0; jp < pp[a + 1] - pp[a]; ++jp) proj_pairs[fill[pp[a] + jp]++] = pair_row[q] + jp;
      }
    }
    if (ent_t.empty()) {
      ent_t.push_back(0);
      ent_beta.push_back(T(0));
    }
    int maxpt = 0, maxpv = 0, maxtv = 0;
    for (int64_t k = 0; k < ntiles; ++k) {
      maxpt = std::max(maxpt, tile_pair_ptr[k + 1] - tile_pair_ptr[k]);
      maxtv = std::max(maxtv, pair_boff[tile_pair_ptr[k + 1]] - pair_boff[tile_pair_ptr[k]]);
    }
    for (int64_t q = 0; q < npairs; ++q) maxpv = std::max(maxpv, pair_boff[q + 1] - pair_boff[q]);
    // LDS: the orbital tile, then as many projector values (and their
    // points) as fit; a batch always holds at least one whole pair
    int dev = 0, maxlds = 0;
    KS_HIP(hipGetDevice(&dev));
    KS_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int P = p->tdim[0] * p->tdim[1] * p->tdim[2];
    const size_t fixed = nl_project_lds(P, sizeof(T), maxpt, 0);
    if (fixed >= (size_t)maxlds) return fail(KS_E_UNSUPPORTED, "too many atoms touch one tile of grid points");
    const int64_t room = (int64_t)(((size_t)maxlds - fixed) / (sizeof(T) + 2)) & ~int64_t(7);
    const int budget = (int)std::min<int64_t>(room, std::max(maxtv, 8));
    if (budget < maxpv) return fail(KS_E_UNSUPPORTED, "one atom's projector values in a tile exceed the LDS");
    p->npairs = npairs;
    p->nrows = nrows;
    p->maxpt = maxpt;
    p->budget = budget;
    if ((rc = upload_vec(tile_pair_ptr, &p->tile_pair_ptr))) return rc;
    if ((rc = upload_vec(pair_ent_ptr, &p->pair_ent_ptr))) return rc;
    if ((rc = upload_vec(pair_boff, &p->pair_boff))) return rc;
    if ((rc = upload_vec(pair_row, &p->pair_row))) return rc;
    if ((rc = upload_vec(ent_t, &p->ent_t))) return rc;
    T* eb2 = nullptr;
    if ((rc = upload_vec(ent_beta, &eb2))) return rc;
    p->ent_beta = eb2;
    if ((rc = upload_vec(proj_pair_ptr, &p->proj_pair_ptr))) return rc;
    if ((rc = upload_vec(proj_pairs, &p->proj_pairs))) return rc;
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

// M = D Y (rows scaled), written in the block precision.  Y = L^-H from the
// deflating Cholesky has zero rows and columns for dead columns, so those
// columns of the orthonormalised block are exactly zero.
template <typename T>
__global__ void k_cholqr_coef(const double2* __restrict__ Y, int ldy, int n, const double* __restrict__ dvec,
                              c2<T>* __restrict__ M, int ldm) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double2 y = Y[i + (int64_t)j * ldy];
    M[i + (int64_t)j * ldm] = cmake<c2<T>>((T)(dvec[i] * y.x), (T)(dvec[i] * y.y));
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
// Buffers of the residual + preconditioner stage besides its FFT scratch
// block: partial sums and kinetic energies (TPA), and the learned network's
// band chunk (inputs, activations, outputs, non-finite flags, column norms).
struct PrecondWs {
  double* partial = nullptr;
  double* E = nullptr;
  int cnn_chunk = 0;
  float* cnn_x = nullptr;    // chunk x 3 x Ng
  float* cnn_buf = nullptr;  // chunk x 32 x Ng
  float* cnn_y = nullptr;    // chunk x 2 x Ng
  int32_t* cnn_bad = nullptr;
  double* cnn_norm = nullptr;  // nb column norms of the TPA output
  double* cnn_part = nullptr;  // column-norm partial sums of one chunk
};

static char* precond_layout(const ks_plan& p, char* q, int nb, bool cnn, PrecondWs& w) {
  auto take = [&](size_t bytes) { char* r = q; q += al(bytes); return r; };
  const int n0 = p.fft.ax[0].n, n1 = p.fft.ax[1].n, n2 = p.fft.ax[2].n;
  const size_t cnt = std::max<size_t>((size_t)std::max(n0, p.a_parts), (size_t)n1 * (n2 / p.zc));
  w.partial = reinterpret_cast<double*>(take((size_t)nb * cnt * 8));
  w.E = reinterpret_cast<double*>(take((size_t)nb * 8));
  if (cnn) {
    w.cnn_chunk = std::min(nb, 32);
    w.cnn_x = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 3 * p.Ng * 4));
    w.cnn_buf = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 32 * p.Ng * 4));
    w.cnn_y = reinterpret_cast<float*>(take((size_t)w.cnn_chunk * 2 * p.Ng * 4));
    w.cnn_bad = reinterpret_cast<int32_t*>(take((size_t)w.cnn_chunk * 4));
    w.cnn_norm = reinterpret_cast<double*>(take((size_t)nb * 8));
    w.cnn_part = reinterpret_cast<double*>(take(column_norms_partial(w.cnn_chunk) * 8));
  }
  return q;
}

// ks_precond_apply's workspace: the FFT scratch block, then PrecondWs.
static size_t precond_full_work_bytes(const ks_plan& p, int nb, bool cnn) {
  static char probe alignas(256);
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  PrecondWs w;
  char* end = precond_layout(p, &probe + al((size_t)p.Ng * nb * es), nb, cnn, w);
  return (size_t)(end - &probe);
}

struct LobWs {
  double2* S;   // m x m
  double2* H;
  double2* C;   // m x nb (FP64)
  void* Cb;     // m x nb block precision
  double2* G;   // nb x nb
  double2* S22; // (m - nb)^2: the [W P] block of S, kept for the next P's Gram
  double2* T22; // (m - nb) x nb
  double2* Y;   // nb x nb
  void* M;      // nb x nb block precision
  double* dvec; // nb
  double* wnew; // m
  int32_t* info;  // 4 ints of scratch
  void* summary;  // theta, res (nb doubles each) and the status words, packed for one read
  void* dc;
  void* gram;
  void* hegv;
  void* potrf;
  double2* ttmp;
  PrecondWs pw;
  char* end;
};

static size_t summary_bytes(int nb) { return (size_t)16 * nb + KS_STATUS_WORDS * 4; }

static LobWs lob_ws(const ks_plan& p, void* work, int nb) {
  const int m = 3 * nb;
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  char* q = static_cast<char*>(work);
  LobWs w;
  auto take = [&](size_t bytes) { char* r = q; q += al(bytes); return r; };
  w.S = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.H = reinterpret_cast<double2*>(take((size_t)m * m * 16));
  w.C = reinterpret_cast<double2*>(take((size_t)m * nb * 16));
  w.Cb = take((size_t)m * nb * es);
  w.G = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
  w.S22 = reinterpret_cast<double2*>(take((size_t)(m - nb) * (m - nb) * 16));
  w.T22 = reinterpret_cast<double2*>(take((size_t)(m - nb) * nb * 16));
  w.Y = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
  w.M = take((size_t)nb * nb * es);
  w.dvec = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.wnew = reinterpret_cast<double*>(take((size_t)m * 8));
  w.info = reinterpret_cast<int32_t*>(take(16));
  w.summary = take(summary_bytes(nb));
  w.dc = take(nl_dc_bytes(p, nb));
  w.gram = take(gram_work_bytes(m, p.Ng));
  w.hegv = take(hegv_work(m, nb));
  w.potrf = take(potrf_work(nb));
  w.ttmp = reinterpret_cast<double2*>(take((size_t)32 * std::max(nb, 1) * 16));
  q = precond_layout(p, q, nb, true, w.pw);
  w.end = q;
  return w;
}

static size_t lobpcg_work_bytes(const ks_plan& p, int nb) {
  // lay the buffers out from a dummy aligned base and measure the span
  static char probe alignas(256);
  LobWs w = lob_ws(p, &probe, nb);
  return (size_t)(w.end - &probe);
}

// ks_subspace_sin's workspace
struct AngleWs {
  double2* G;  // k x k
  double2* M;  // k x k
  double2* S;  // k x k identity
  double2* C;  // k
  double* w;
  int32_t* info;
  void* gram;
  void* hegv;
  char* end;
};

static AngleWs angle_ws(const ks_plan& p, void* work, int k) {
  char* q = static_cast<char*>(work);
  AngleWs w;
  auto take = [&](size_t bytes) { char* r = q; q += al(bytes); return r; };
  w.G = reinterpret_cast<double2*>(take((size_t)k * k * 16));
  w.M = reinterpret_cast<double2*>(take((size_t)k * k * 16));
  w.S = reinterpret_cast<double2*>(take((size_t)k * k * 16));
  w.C = reinterpret_cast<double2*>(take((size_t)k * 16));
  w.w = reinterpret_cast<double*>(take(8));
  w.info = reinterpret_cast<int32_t*>(take(16));
  w.gram = take(gram_work_bytes(k, p.Ng));
  w.hegv = take(hegv_work(k, 1));
  w.end = q;
  return w;
}

static size_t angle_work_bytes(const ks_plan& p, int k) {
  static char probe alignas(256);
  return (size_t)(angle_ws(p, &probe, k).end - &probe);
}

__global__ void k_sin_from_sigma2(const double* __restrict__ w, const int32_t* __restrict__ info,
                                  double* __restrict__ out) {
  if (threadIdx.x == 0) *out = *info != 0 ? __longlong_as_double(0x7ff8000000000000ll) : sqrt(fmax(0.0, 1.0 - *w));
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

template <typename T>
static int subspace_sin(const ks_plan& p, const void* A, const void* B, int64_t ld, int k, double* out, void* work,
                        hipStream_t s) {
  AngleWs w = angle_ws(p, work, k);
  int rc;
  auto LA = blist<T>(A, nullptr, nullptr, ld, k);
  auto LB = blist<T>(B, nullptr, nullptr, ld, k);
  if ((rc = gram_general<T>(LA, LB, k, p.Ng, w.G, k, w.gram, s))) return rc;
  if ((rc = zgemm('C', 'N', k, k, k, 1.0, w.G, k, w.G, k, 0.0, w.M, k, s))) return rc;
  hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)k * k)), dim3(256), 0, s, w.S, k, k);
  if ((rc = hegv(k, 1, w.M, k, w.S, k, w.w, w.C, k, w.hegv, w.info, nullptr, s))) return rc;
  hipLaunchKernelGGL(k_sin_from_sigma2, dim3(1), dim3(64), 0, s, w.w, w.info, out);
  KS_LAUNCH_CHECK("subspace_sin");
  return 0;
}

__global__ void k_status_clear(int32_t* __restrict__ st) {
  if (threadIdx.x < KS_STATUS_WORDS) st[threadIdx.x] = 0;
}

// Flags of the step from its counters, the subspace solve's info and the
// finiteness of theta and res (res may be null); then theta, res and the
// status words packed into `summary` for one device-to-host copy.
__global__ void __launch_bounds__(256)
k_finish_status(int32_t* __restrict__ st, const double* __restrict__ theta, const double* __restrict__ res, int nb,
                unsigned char* __restrict__ summary) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int my = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const double t = theta[i];
    if (!isfinite(t) || (res && !isfinite(res[i]))) my = 1;
  }
  if (my) atomicOr(&bad, 1);
  __syncthreads();
  double* sd = reinterpret_cast<double*>(summary);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    sd[i] = theta[i];
    sd[nb + i] = res ? res[i] : 0.0;
  }
  if (threadIdx.x == 0) {
    int f = 0;
    if (st[KS_ST_DEAD_W] + st[KS_ST_DEAD_P] + st[KS_ST_DEAD_BASIS] + st[KS_ST_DEAD_X] > 0) f |= KS_FLAG_DEFLATED;
    if (st[KS_ST_INFO] != 0) f |= KS_FLAG_SOLVE_FAILED;
    if (bad) f |= KS_FLAG_NONFINITE;
    st[KS_ST_FLAGS] = f;
    int32_t* si = reinterpret_cast<int32_t*>(sd + 2 * nb);
    for (int k = 0; k < KS_STATUS_WORDS; ++k) si[k] = st[k];
  }
}

// B <- B D L^-H (columns scaled to unit norm, then Cholesky-QR), written to
// out.  The Cholesky deflates: a column that depends numerically on the
// ones before it becomes an exactly-zero column (counted in *ndead).  No
// host synchronisation.
// gram_in: B's Gram matrix (nb x nb, FP64) when the caller has it; else it
// is formed from B.
template <typename T>
static int block_orthonormalise(const ks_plan& p, const LobWs& w, const void* B, void* out, int64_t ld, int nb,
                                const double* res, double lock_tol, int32_t* ndead, hipStream_t s,
                                const double2* gram_in = nullptr) {
  int rc;
  auto L1 = blist<T>(B, nullptr, nullptr, ld, nb);
  if (gram_in != nullptr) {
    KS_HIP(hipMemcpyAsync(w.G, gram_in, (size_t)nb * nb * sizeof(double2), hipMemcpyDeviceToDevice, s));
  } else if ((rc = gram<T>(L1, L1, nullptr, nb, p.Ng, w.G, nb, nullptr, 0, w.gram, s))) {
    return rc;
  }
  hipLaunchKernelGGL(k_colscale, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, w.G, nb, nb, res, lock_tol,
                     w.dvec);
  hipLaunchKernelGGL(k_scale_gram, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.G, nb, nb, w.dvec);
  KS_LAUNCH_CHECK("colscale");
  if ((rc = potrf_deflate(nb, w.G, nb, w.potrf, w.info + 1, ndead, s))) return rc;
  hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb);
  if ((rc = trsm('C', nb, nb, w.G, nb, w.Y, nb, w.potrf, w.ttmp, w.info + 1, s))) return rc;
  hipLaunchKernelGGL((k_cholqr_coef<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb, w.dvec,
                     static_cast<c2<T>*>(w.M), nb);
  KS_LAUNCH_CHECK("cholqr_coef");
  const auto* M = static_cast<const c2<T>*>(w.M);
  // D L^-H is upper triangular
  return rotate<T>(L1, nb, nb, M, nb, nb, p.Ng, static_cast<c2<T>*>(out), nullptr, ld, s, true);
}

// Residual, norms and preconditioned residual W (lock-masked), for every
// preconditioner kind: the learned ones run the network on the residual
// (KS_PRECOND_CNN) or on the TPA output with the skip connection
// (KS_PRECOND_CNN_TPA), in band chunks.  tmp: one Ng x nb scratch block.
template <typename T>
static int precond_full(const ks_plan& p, int kind_full, double lock_tol, const float* cnn_params, const T* v,
                        const c2<T>* X, const c2<T>* AX, const double* theta, int64_t ld, int nb, c2<T>* W,
                        double* res, c2<T>* tmp, const PrecondWs& pw, hipStream_t s) {
  const bool learned = kind_full == KS_PRECOND_CNN || kind_full == KS_PRECOND_CNN_TPA;
  const int kind = kind_full == KS_PRECOND_CNN ? KS_PRECOND_NONE
                   : kind_full == KS_PRECOND_CNN_TPA ? KS_PRECOND_TPA
                                                     : kind_full;
  int rc;
  if ((rc = precond_apply<T>(p, kind, X, AX, theta, ld, nb, lock_tol, W, res, tmp, pw.partial, pw.E, s))) return rc;
  if (!learned) return 0;
  const bool skip = kind_full == KS_PRECOND_CNN_TPA;
  for (int b0 = 0; b0 < nb; b0 += pw.cnn_chunk) {
    const int nc = std::min(pw.cnn_chunk, nb - b0);
    c2<T>* R = W + (int64_t)b0 * ld;
    const double* nrm = res + b0;
    if (skip) {
      if ((rc = column_norms<T>(R, ld, nc, p.Ng, pw.cnn_part, pw.cnn_norm + b0, s))) return rc;
      nrm = pw.cnn_norm + b0;
    }
    if ((rc = cnn_input_impl<T>(p, R, ld, nrm, v, theta + b0, nc, pw.cnn_x, s))) return rc;
    if ((rc = cnn_infer_impl(p, cnn_params, nc, pw.cnn_x, pw.cnn_y, pw.cnn_buf, s))) return rc;
    if (skip && (rc = cnn_skip_impl(p, nc, pw.cnn_x, pw.cnn_y, s))) return rc;
    if ((rc = cnn_output_impl<T>(p, pw.cnn_y, nc, res + b0, lock_tol, pw.cnn_bad, R, ld, s))) return rc;
  }
  return 0;
}

// theta <- the new Ritz values, status flags, and (with a host summary
// buffer) the one device-to-host copy of the step, then a wait for it.
static int finish_step(const LobWs& w, ks_lobpcg_state* st, const double* res, int nb, hipStream_t s) {
  KS_HIP(hipMemcpyAsync(st->theta, w.wnew, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_finish_status, dim3(1), dim3(256), 0, s, st->status, st->theta, res, nb,
                     static_cast<unsigned char*>(w.summary));
  KS_LAUNCH_CHECK("finish_status");
  if (st->host_summary) {
    KS_HIP(hipMemcpyAsync(st->host_summary, w.summary, summary_bytes(nb), hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
  }
  return 0;
}

template <typename T>
static int lob_init(const ks_plan& p, const void* v, ks_lobpcg_state* st, void* work, hipStream_t s) {
  const int nb = st->nb;
  const int64_t ld = st->ld;
  LobWs w = lob_ws(p, work, nb);
  int rc;
  hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, s, st->status);
  // Cholesky-QR of the start block (a dependent column would become zero)
  auto LX = blist<T>(st->X, nullptr, nullptr, ld, nb);
  if ((rc = gram<T>(LX, LX, nullptr, nb, p.Ng, w.G, nb, nullptr, 0, w.gram, s))) return rc;
  if ((rc = potrf_deflate(nb, w.G, nb, w.potrf, w.info + 1, st->status + KS_ST_DEAD_X, s))) return rc;
  hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb, nb);
  if ((rc = trsm('C', nb, nb, w.G, nb, w.Y, nb, w.potrf, w.ttmp, w.info + 1, s))) return rc;
  hipLaunchKernelGGL((k_to_block<T>), dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, s, w.Y, nb,
                     static_cast<c2<T>*>(w.M), nb, nb, nb);
  KS_LAUNCH_CHECK("to_block");
  if ((rc = rotate<T>(LX, nb, nb, static_cast<const c2<T>*>(w.M), nb, nb, p.Ng, static_cast<c2<T>*>(st->Xn), nullptr,
                      ld, s, true)))
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
  if ((rc = hegv(nb, nb, w.H, nb, w.S, nb, w.wnew, w.C, nb, w.hegv, st->status + KS_ST_INFO,
                 st->status + KS_ST_DEAD_BASIS, s)))
    return rc;
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
  st->has_p = 0;
  st->p_gram_ok = 0;
  st->iter = 0;
  return finish_step(w, st, nullptr, nb, s);
}

template <typename T>
static int lob_step(const ks_plan& p, const void* v, ks_lobpcg_state* st, const ks_lobpcg_opts* o, void* work,
                    hipStream_t s) {
  const int nb = st->nb;
  const int64_t ld = st->ld;
  LobWs w = lob_ws(p, work, nb);
  int rc;
  using T2 = c2<T>;
  hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, s, st->status);
  // 1. residual, its norms, preconditioned and lock-masked W (into Xn)
  if ((rc = precond_full<T>(p, o->precond, o->lock_tol, o->cnn_params, static_cast<const T*>(v),
                            static_cast<const T2*>(st->X), static_cast<const T2*>(st->AX), st->theta, ld, nb,
                            static_cast<T2*>(st->Xn), st->res, static_cast<T2*>(st->T1), w.pw, s)))
    return rc;
  // 2. W <- W - X (X^H W), then W <- W D L^-H
  if ((rc = project_out<T>(static_cast<const T2*>(st->X), static_cast<const T2*>(st->Xn), static_cast<T2*>(st->W), ld,
                           nb, p.Ng, w.G, w.Cb, w.gram, s)))
    return rc;
  if ((rc = block_orthonormalise<T>(p, w, st->W, st->Xn, ld, nb, nullptr, 0.0, st->status + KS_ST_DEAD_W, s)))
    return rc;
  std::swap(st->W, st->Xn);
  // 3. AW = H W; soft-locked bands (res <= lock_tol) have exactly zero W
  // columns (masked in step 1, kept zero by the projection and dropped by
  // the deflating Cholesky-QR), so their transforms are skipped
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->W), ld, static_cast<T2*>(st->AW), ld,
                       nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s, st->res, o->lock_tol)))
    return rc;
  // 4. P, AP masked and orthonormalised
  if (st->has_p) {
    if ((rc = block_orthonormalise<T>(p, w, st->P, st->Pn, ld, nb, st->res, o->lock_tol, st->status + KS_ST_DEAD_P,
                                      s, st->p_gram_ok ? static_cast<const double2*>(st->p_gram) : nullptr)))
      return rc;
    std::swap(st->P, st->Pn);
    // the same mask zeroed the locked P columns
    if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->P), ld, static_cast<T2*>(st->AP), ld,
                         nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s, st->res, o->lock_tol)))
      return rc;
  }
  // 5. subspace matrices
  const int m = st->has_p ? 3 * nb : 2 * nb;
  auto LV = blist<T>(st->X, st->W, st->P, ld, nb);
  auto LAV = blist<T>(st->AX, st->AW, st->AP, ld, nb);
  {
    TimerScope tb(KF_GRAM_BASIS, s);
    if ((rc = gram<T>(LV, LV, &LAV, m, p.Ng, w.S, m, w.H, m, w.gram, s))) return rc;
  }
  hipLaunchKernelGGL(k_decouple, dim3(1), dim3(256), 0, s, w.S, m, w.H, m, m);
  KS_LAUNCH_CHECK("decouple");
  // the [W P] block of S, before the factorisation overwrites it.  FP64
  // plans only: a mixed plan's P is rotated in FP32 (and by FP32
  // coefficients), so its computed Gram departs from C^H S C by the FP32
  // rounding, which the Cholesky-QR of a nearly dependent P magnifies; it
  // forms P's Gram from P itself.
  const int m2 = m - nb;
  const bool carry = st->p_gram != nullptr && p.prec == KS_FP64;
  if (carry)
    KS_HIP(hipMemcpy2DAsync(w.S22, (size_t)m2 * sizeof(double2), w.S + nb + (int64_t)nb * m,
                            (size_t)m * sizeof(double2), (size_t)m2 * sizeof(double2), (size_t)m2,
                            hipMemcpyDeviceToDevice, s));
  // 6. reduction and eigensolve; basis vectors that depend numerically on
  // earlier ones are dropped by the deflating Cholesky
  if ((rc = hegv(m, nb, w.H, m, w.S, m, w.wnew, w.C, m, w.hegv, st->status + KS_ST_INFO,
                 st->status + KS_ST_DEAD_BASIS, s)))
    return rc;
  // the next P = V_[W P] C_[W P] has Gram C_[W P]^H S_[W P] C_[W P] (dead
  // basis vectors have zero coefficients, so their decoupled entries of S
  // contribute nothing)
  st->p_gram_ok = 0;
  if (carry) {
    if ((rc = zgemm('N', 'N', m2, nb, m2, 1.0, w.S22, m2, w.C + nb, m, 0.0, w.T22, m2, s))) return rc;
    if ((rc = zgemm('C', 'N', nb, nb, m2, 1.0, w.C + nb, m, w.T22, m2, 0.0, static_cast<double2*>(st->p_gram), nb,
                    s)))
      return rc;
    st->p_gram_ok = 1;
  }
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
    if ((rc = block_orthonormalise<T>(p, w, st->X, st->Xn, ld, nb, nullptr, 0.0, st->status + KS_ST_DEAD_X, s)))
      return rc;
    std::swap(st->X, st->Xn);
  }
  // 9. AX by a fresh H-apply (AP is formed the same way next step)
  if ((rc = apply_h<T>(p, static_cast<const T*>(v), static_cast<const T2*>(st->X), ld, static_cast<T2*>(st->AX), ld,
                       nb, static_cast<T2*>(st->T1), static_cast<T2*>(w.dc), s)))
    return rc;
  st->has_p = 1;
  st->iter += 1;
  return finish_step(w, st, st->res, nb, s);
}

// The projector set's CSR structure, checked on the host before any table
// is built from it: both atom pointer arrays start at 0, never decrease and
// end at the totals; every value block has |S_a| * p_a entries; support
// indices lie on the grid; at most 9 projectors per atom (the widest
// projection kernel).  Returns the reason, or nullptr when valid.
static const char* check_projset(const ks_projset& ps, int64_t Ng) {
  if (ps.n_atoms < 0 || ps.n_proj < 0 || ps.n_supp < 0) return "negative projector set sizes";
  const int32_t* sp = ps.atom_supp_ptr;
  const int32_t* pp = ps.atom_proj_ptr;
  const int64_t* bp = ps.beta_ptr;
  if (sp[0] != 0 || pp[0] != 0 || bp[0] != 0) return "projector CSR pointers must start at 0";
  for (int a = 0; a < ps.n_atoms; ++a) {
    if (sp[a + 1] < sp[a] || pp[a + 1] < pp[a]) return "projector CSR pointers decrease";
    const int np = pp[a + 1] - pp[a];
    if (np > 9) return "more than 9 projectors per atom";
    if (bp[a + 1] - bp[a] != (int64_t)np * (sp[a + 1] - sp[a]))
      return "beta_ptr does not match |S_a| * projectors of an atom";
  }
  if (pp[ps.n_atoms] != ps.n_proj || sp[ps.n_atoms] != ps.n_supp) return "projector CSR pointers inconsistent";
  for (int64_t i = 0; i < ps.n_supp; ++i)
    if (ps.supp_idx[i] < 0 || ps.supp_idx[i] >= Ng) return "support index out of the grid";
  return nullptr;
}

// A projector set with Bloch phases folded in: projector j of atom a
// becomes the real pair 2j (values b cos(k.d_s)) and 2j + 1 (b sin(k.d_s)),
// d_s the displacement of support point s from the atom; both keep D_j.
struct BlochProjset {
  std::vector<int32_t> pp;
  std::vector<int64_t> bp;
  std::vector<double> beta, D;
  ks_projset ps;
};

static void bloch_projset(const ks_projset& in, const double* disp, const double* k, BlochProjset& o) {
  const int na = in.n_atoms;
  o.pp.assign(na + 1, 0);
  o.bp.assign(na + 1, 0);
  for (int a = 0; a < na; ++a) {
    const int np = in.atom_proj_ptr[a + 1] - in.atom_proj_ptr[a];
    const int64_t ns = in.atom_supp_ptr[a + 1] - in.atom_supp_ptr[a];
    o.pp[a + 1] = o.pp[a] + 2 * np;
    o.bp[a + 1] = o.bp[a] + 2 * np * ns;
  }
  o.beta.assign((size_t)o.bp[na], 0.0);
  o.D.assign((size_t)2 * in.n_proj, 0.0);
  std::vector<double> c, sn;
  for (int a = 0; a < na; ++a) {
    const int np = in.atom_proj_ptr[a + 1] - in.atom_proj_ptr[a];
    const int64_t s0 = in.atom_supp_ptr[a], ns = in.atom_supp_ptr[a + 1] - s0;
    c.resize(ns);
    sn.resize(ns);
    for (int64_t s = 0; s < ns; ++s) {
      const double* d = disp + 3 * (s0 + s);
      const double kd = k[0] * d[0] + k[1] * d[1] + k[2] * d[2];
      c[s] = cos(kd);
      sn[s] = sin(kd);
    }
    for (int j = 0; j < np; ++j) {
      const double* src = in.beta + in.beta_ptr[a] + (int64_t)j * ns;
      double* dc = o.beta.data() + o.bp[a] + (int64_t)(2 * j) * ns;
      double* ds = dc + ns;
      for (int64_t s = 0; s < ns; ++s) {
        dc[s] = src[s] * c[s];
        ds[s] = src[s] * sn[s];
      }
      const int P = in.atom_proj_ptr[a] + j;
      o.D[2 * P] = o.D[2 * P + 1] = in.D[P];
    }
  }
  o.ps = in;
  o.ps.n_proj = 2 * in.n_proj;
  o.ps.atom_proj_ptr = o.pp.data();
  o.ps.beta_ptr = o.bp.data();
  o.ps.beta = o.beta.data();
  o.ps.D = o.D.data();
}

static int plan_create(ks_plan** out, const ks_grid* grid, const double* kvec, const ks_projset* proj,
                       const double* supp_disp, int32_t nb_max, int32_t precision, void* stream);

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
  return plan_create(out, grid, nullptr, proj, nullptr, nb_max, precision, stream);
}

int ks_plan_create_k(ks_plan** out, const ks_grid* grid, const double* kvec, const ks_projset* proj,
                     const double* supp_disp, int32_t nb_max, int32_t precision, void* stream) {
  g_last_error.clear();
  if (!kvec) return fail(-3, "kvec is null");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(kvec[a])) return fail(-3, "kvec must be finite");
  const bool nonzero = kvec[0] != 0.0 || kvec[1] != 0.0 || kvec[2] != 0.0;
  if (nonzero && proj && proj->n_proj > 0 && !supp_disp) return fail(-5, "supp_disp is null");
  return plan_create(out, grid, nonzero ? kvec : nullptr, proj, supp_disp, nb_max, precision, stream);
}

}  // extern "C"

namespace ks {

static int plan_create(ks_plan** out, const ks_grid* grid, const double* kvec, const ks_projset* proj,
                       const double* supp_disp, int32_t nb_max, int32_t precision, void* stream) {
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
    p->fft.kvec[a] = kvec ? kvec[a] : 0.0;
    p->Ng *= grid->n[a];
  }
  p->fft.skip_res = nullptr;
  p->fft.skip_tol = 0.0;
  // the projector set is checked before any device work
  if (proj && proj->n_proj > 0) {
    const char* why = nullptr;
    if (!proj->atom_supp_ptr || !proj->supp_idx || !proj->atom_proj_ptr || !proj->beta_ptr || !proj->beta || !proj->D)
      why = "projector set has null arrays";
    else
      why = check_projset(*proj, p->Ng);
    if (why) {
      delete p;
      return fail(-3, why);
    }
    if (kvec)
      for (int a = 0; a < proj->n_atoms; ++a)
        if (2 * (proj->atom_proj_ptr[a + 1] - proj->atom_proj_ptr[a]) > 9) {
          delete p;
          return fail(KS_E_UNSUPPORTED, "a plan with a Bloch vector takes at most 4 projectors per atom (s and p)");
        }
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
  p->a_parts = n0;
  if (p->lds_plane > (size_t)maxlds) {
    // split planes: the largest row and column groups of at most 4096
    // points (16 per thread of a 256-thread block) that fit in the LDS
    p->split = 1;
    for (int r = 1; r <= n1; ++r)
      if (n1 % r == 0 && (int64_t)r * n2 <= 4096 && (size_t)(r * n2 + n2) * es <= (size_t)maxlds) p->ry = r;
    for (int z = 1; z <= n2; ++z)
      if (n2 % z == 0 && (int64_t)n1 * z <= 4096 && (size_t)(n1 * z + n1) * es <= (size_t)maxlds) p->zc2 = z;
    p->lds_rows = (size_t)(p->ry * n2 + n2) * es;
    p->lds_cols = (size_t)(n1 * p->zc2 + n1) * es;
    p->a_parts = p->ry > 0 ? n0 * (n1 / p->ry) : 0;
  }
  if ((p->split && (p->ry == 0 || p->zc2 == 0)) || p->lds_pencil > (size_t)maxlds) {
    delete p;
    return fail(KS_E_UNSUPPORTED, "plane does not fit in LDS");
  }
  int rc = 0;
  for (int a = 0; a < 3 && rc == 0; ++a)
    rc = precision == KS_FP64 ? upload_twiddles<double>(grid->n[a], &p->tw[a]) : upload_twiddles<float>(grid->n[a], &p->tw[a]);
  if (rc == 0 && proj && proj->n_proj > 0) {
    const ks_projset* use = proj;
    BlochProjset bl;
    if (kvec) {
      bloch_projset(*proj, supp_disp, kvec, bl);
      use = &bl.ps;
      p->kpairs = 1;
    }
    rc = precision == KS_FP64 ? upload_proj<double>(p, use) : upload_proj<float>(p, use);
  }
  if (rc) {
    ks_plan_destroy(p);
    return rc;
  }
  KS_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  *out = p;
  return 0;
}

}  // namespace ks

extern "C" {

int ks_plan_destroy(ks_plan* p) {
  if (!p) return 0;
  for (int a = 0; a < 3; ++a) (void)hipFree(p->tw[a]);
  void* bufs[] = {p->Dcoef,         p->blk_ptr,      p->blk_proj, p->ell_ptr,   p->ell_lp,
                  p->ell_beta,      p->tile_pair_ptr, p->pair_ent_ptr, p->pair_boff, p->pair_row,
                  p->ent_t,         p->ent_beta,     p->proj_pair_ptr, p->proj_pairs};
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
    case KS_OP_PRECOND: *bytes = precond_full_work_bytes(*p, nb, false); return 0;
    case KS_OP_PRECOND_CNN: *bytes = precond_full_work_bytes(*p, nb, true); return 0;
    case KS_OP_ANGLE: *bytes = angle_work_bytes(*p, nb); return 0;
    case KS_OP_SCF: *bytes = scf_work_bytes(*p); return 0;
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
  char* dc = tmp + al((size_t)p->Ng * nb * es);  // coefficients, then projection partials
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return apply_h<double>(*p, static_cast<const double*>(v_loc), static_cast<const double2*>(psi), ld_psi,
                           static_cast<double2*>(hpsi), ld_hpsi, nb, reinterpret_cast<double2*>(tmp),
                           reinterpret_cast<double2*>(dc), s);
  return apply_h<float>(*p, static_cast<const float*>(v_loc), static_cast<const float2*>(psi), ld_psi,
                        static_cast<float2*>(hpsi), ld_hpsi, nb, reinterpret_cast<float2*>(tmp),
                        reinterpret_cast<float2*>(dc), s);
}

int ks_precond_apply(const ks_plan* p, const ks_lobpcg_opts* opts, const void* v_loc, const void* X, const void* AX,
                     const double* theta, int64_t ld, int32_t nb, void* W, double* res, void* work, size_t work_bytes,
                     void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!opts) return fail(-2, "opts is null");
  const int kind = opts->precond;
  if (kind != KS_PRECOND_NONE && kind != KS_PRECOND_TPA && kind != KS_PRECOND_CNN && kind != KS_PRECOND_CNN_TPA)
    return fail(-2, "unknown preconditioner");
  const bool learned = kind == KS_PRECOND_CNN || kind == KS_PRECOND_CNN_TPA;
  if (learned && !opts->cnn_params) return fail(-2, "CNN preconditioner without parameters");
  if (learned && !v_loc) return fail(-3, "v_loc is null (the learned kinds read the local potential)");
  if (!X) return fail(-4, "X is null");
  if (!AX) return fail(-5, "AX is null");
  if (!theta) return fail(-6, "theta is null");
  if (ld < p->Ng) return fail(-7, "ld < Ng");
  if (nb <= 0 || nb > p->nb_max) return fail(-8, "nb out of range");
  if (!W) return fail(-9, "W is null");
  if (!res) return fail(-10, "res is null");
  if (!work) return fail(-11, "work is null");
  if (work_bytes < precond_full_work_bytes(*p, nb, learned)) return fail(KS_E_WORKSPACE, "workspace too small");
  const size_t es = p->prec == KS_FP64 ? 16 : 8;
  char* tmp = static_cast<char*>(work);
  PrecondWs pw;
  precond_layout(*p, tmp + al((size_t)p->Ng * nb * es), nb, learned, pw);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->prec == KS_FP64)
    return precond_full<double>(*p, kind, opts->lock_tol, opts->cnn_params, static_cast<const double*>(v_loc),
                                static_cast<const double2*>(X), static_cast<const double2*>(AX), theta, ld, nb,
                                static_cast<double2*>(W), res, reinterpret_cast<double2*>(tmp), pw, s);
  return precond_full<float>(*p, kind, opts->lock_tol, opts->cnn_params, static_cast<const float*>(v_loc),
                             static_cast<const float2*>(X), static_cast<const float2*>(AX), theta, ld, nb,
                             static_cast<float2*>(W), res, reinterpret_cast<float2*>(tmp), pw, s);
}

int ks_subspace_sin(const ks_plan* p, const void* A, const void* B, int64_t ld, int32_t k, double* sin_max,
                    void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!A) return fail(-2, "A is null");
  if (!B) return fail(-3, "B is null");
  if (ld < p->Ng) return fail(-4, "ld < Ng");
  if (k <= 0 || k > p->nb_max) return fail(-5, "k out of range");
  if (!sin_max) return fail(-6, "sin_max is null");
  if (!work) return fail(-7, "work is null");
  if (work_bytes < angle_work_bytes(*p, k)) return fail(KS_E_WORKSPACE, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->prec == KS_FP64 ? subspace_sin<double>(*p, A, B, ld, k, sin_max, work, s)
                            : subspace_sin<float>(*p, A, B, ld, k, sin_max, work, s);
}

// ---------------------------------------------------------------- no-allocation dense solve
// The workspace of hegv_reduce_solve_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only stands for the symbol): the
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[KS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[KS_NOALLOC_MAX_DEVICES] = {};

static int scratch_address(void** out) {
  int dev = 0;
  KS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= KS_NOALLOC_MAX_DEVICES) return fail(KS_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(KS_E_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

int hegv_reduce_solve_noalloc(int32_t n, int32_t nev, void* H, int32_t ldh, void* S, int32_t lds, double* w, void* C,
                              int32_t ldc, int32_t* info_dev, void* stream) {
  g_last_error.clear();
  if (n <= 0 || n > KS_NOALLOC_MAX_N)
    return fail(-1, "n out of range for the no-allocation solve (1.." + std::to_string(KS_NOALLOC_MAX_N) + ")");
  if (nev <= 0 || nev > n) return fail(-2, "nev out of range");
  if (!H) return fail(-3, "H is null");
  if (ldh < n) return fail(-4, "ldh < n");
  if (!S) return fail(-5, "S is null");
  if (lds < n) return fail(-6, "lds < n");
  if (!w) return fail(-7, "w is null");
  if (!C) return fail(-8, "C is null");
  if (ldc < n) return fail(-9, "ldc < n");
  if (!info_dev) return fail(-10, "info is null");
  if (hegv_work(n, nev) > (size_t)KS_NOALLOC_SCRATCH_BYTES)
    return fail(KS_E_WORKSPACE, "workspace of this size exceeds the static scratch array");
  void* work = nullptr;
  int rc = scratch_address(&work);
  if (rc) return rc;
  // the solve reads no workspace value before writing it (its counters and
  // masks are set by its own first kernels), so the previous call's
  // contents need no clearing
  g_timers_suppressed = true;
  rc = hegv(n, nev, static_cast<double2*>(H), ldh, static_cast<double2*>(S), lds, w, static_cast<double2*>(C), ldc,
            work, info_dev, nullptr, static_cast<hipStream_t>(stream));
  g_timers_suppressed = false;
  return rc;
}

int ks_density(const ks_plan* p, const void* X, int64_t ld, int32_t nocc, const double* occ, double* n,
               void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!X) return fail(-2, "X is null");
  if (ld < p->Ng) return fail(-3, "ld < Ng");
  if (nocc <= 0 || nocc > p->nb_max) return fail(-4, "nocc out of range");
  if (!n) return fail(-6, "n is null");
  return density_impl(*p, X, ld, nocc, occ, n, static_cast<hipStream_t>(stream));
}

int ks_hartree(const ks_plan* p, const double* n, double* v_h, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!n) return fail(-2, "n is null");
  if (!v_h) return fail(-3, "v_h is null");
  if (!work) return fail(-4, "work is null");
  if (work_bytes < scf_work_bytes(*p)) return fail(KS_E_WORKSPACE, "workspace too small");
  return hartree_impl(*p, n, v_h, work, static_cast<hipStream_t>(stream));
}

int ks_lda_xc(const ks_plan* p, const double* n, double* v_xc, double* e_xc, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!n) return fail(-2, "n is null");
  if (!v_xc) return fail(-3, "v_xc is null");
  return lda_impl(*p, n, v_xc, e_xc, static_cast<hipStream_t>(stream));
}

int ks_scf_potential(const ks_plan* p, const double* n, const double* v_ion, void* v_eff, double* terms, void* work,
                     size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!n) return fail(-2, "n is null");
  if (!v_ion) return fail(-3, "v_ion is null");
  if (!v_eff) return fail(-4, "v_eff is null");
  if (!terms) return fail(-5, "terms is null");
  if (!work) return fail(-6, "work is null");
  if (work_bytes < scf_work_bytes(*p)) return fail(KS_E_WORKSPACE, "workspace too small");
  return scf_potential_impl(*p, n, v_ion, v_eff, terms, work, static_cast<hipStream_t>(stream));
}

int ks_mix_density(const ks_plan* p, double alpha, const double* n_in, const double* n_out, double* n_next,
                   double* resid, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (!p) return fail(-1, "plan is null");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(-2, "alpha must lie in [0, 1]");
  if (!n_in) return fail(-3, "n_in is null");
  if (!n_out) return fail(-4, "n_out is null");
  if (!n_next) return fail(-5, "n_next is null");
  if (!resid) return fail(-6, "resid is null");
  if (!work) return fail(-7, "work is null");
  if (work_bytes < scf_work_bytes(*p)) return fail(KS_E_WORKSPACE, "workspace too small");
  return mix_impl(*p, alpha, n_in, n_out, n_next, resid, work, static_cast<hipStream_t>(stream));
}

int ks_gram_workspace_size(int64_t K, int32_t m, size_t* bytes) {
  if (K <= 0) return fail(-1, "K must be positive");
  if (m <= 0) return fail(-2, "m must be positive");
  if (!bytes) return fail(-3, "bytes is null");
  *bytes = gram_work_bytes(m, K);
  return 0;
}

int ks_gram_general(int32_t precision, int64_t K, int32_t m, const void* A, const void* B, int64_t ld, void* G,
                    int32_t ldg, void* work, size_t work_bytes, void* stream) {
  g_last_error.clear();
  if (precision != KS_FP64 && precision != KS_MIXED_FP32) return fail(-1, "precision must be KS_FP64 or KS_MIXED_FP32");
  if (K <= 0) return fail(-2, "K must be positive");
  if (m <= 0) return fail(-3, "m must be positive");
  if (!A) return fail(-4, "A is null");
  if (!B) return fail(-5, "B is null");
  if (ld < K) return fail(-6, "ld < K");
  if (!G) return fail(-7, "G is null");
  if (ldg < m) return fail(-8, "ldg < m");
  if (!work) return fail(-9, "work is null");
  if (work_bytes < gram_work_bytes(m, K)) return fail(KS_E_WORKSPACE, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == KS_FP64)
    return gram_general<double>(blist<double>(A, nullptr, nullptr, ld, m), blist<double>(B, nullptr, nullptr, ld, m),
                                m, K, static_cast<double2*>(G), ldg, work, s);
  return gram_general<float>(blist<float>(A, nullptr, nullptr, ld, m), blist<float>(B, nullptr, nullptr, ld, m), m,
                             K, static_cast<double2*>(G), ldg, work, s);
}

int ks_rotate_block(int32_t precision, int64_t K, int32_t m, const void* V, int64_t ld, const void* C, int32_t ldc,
                    int32_t ncol, void* Y, int64_t ldy, void* stream) {
  g_last_error.clear();
  if (precision != KS_FP64 && precision != KS_MIXED_FP32) return fail(-1, "precision must be KS_FP64 or KS_MIXED_FP32");
  if (K <= 0) return fail(-2, "K must be positive");
  if (m <= 0) return fail(-3, "m must be positive");
  if (!V) return fail(-4, "V is null");
  if (ld < K) return fail(-5, "ld < K");
  if (!C) return fail(-6, "C is null");
  if (ldc < m) return fail(-7, "ldc < m");
  if (ncol <= 0) return fail(-8, "ncol must be positive");
  if (!Y) return fail(-9, "Y is null");
  if (ldy < K) return fail(-10, "ldy < K");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == KS_FP64)
    return rotate<double>(blist<double>(V, nullptr, nullptr, ld, m), m, m, static_cast<const double2*>(C), ldc, ncol,
                          K, static_cast<double2*>(Y), nullptr, ldy, s);
  return rotate<float>(blist<float>(V, nullptr, nullptr, ld, m), m, m, static_cast<const float2*>(C), ldc, ncol, K,
                       static_cast<float2*>(Y), nullptr, ldy, s);
}

int hegv_reduce_variant(int32_t variant, int32_t n, const void* H, int32_t ldh, void* S, int32_t lds, void* K,
                        int32_t ldk, void* work, size_t work_bytes, int32_t* info_dev, void* stream) {
  g_last_error.clear();
  if (variant < KS_REDUCE_INVERSE || variant > KS_REDUCE_TWO_SIDED) return fail(-1, "unknown reduction variant");
  if (n <= 0 || n > kHegvMaxN) return fail(-2, "n out of range");
  if (!H) return fail(-3, "H is null");
  if (ldh < n) return fail(-4, "ldh < n");
  if (!S) return fail(-5, "S is null");
  if (lds < n) return fail(-6, "lds < n");
  if (!K) return fail(-7, "K is null");
  if (ldk < n) return fail(-8, "ldk < n");
  if (K == H || K == S) return fail(-7, "K must not alias H or S");
  if (!work) return fail(-9, "work is null");
  if (work_bytes < hegv_work(n, 1)) return fail(KS_E_WORKSPACE, "workspace too small");
  if (!info_dev) return fail(-11, "info is null");
  return reduce_variant(variant, n, static_cast<const double2*>(H), ldh, static_cast<double2*>(S), lds,
                        static_cast<double2*>(K), ldk, work, info_dev, static_cast<hipStream_t>(stream));
}

int sygv_reduce_variant(int32_t variant, int32_t n, const double* H, int32_t ldh, double* S, int32_t lds, double* K,
                        int32_t ldk, void* work, size_t work_bytes, int32_t* info_dev, void* stream) {
  g_last_error.clear();
  if (variant < KS_REDUCE_INVERSE || variant > KS_REDUCE_TWO_SIDED) return fail(-1, "unknown reduction variant");
  if (n <= 0 || n > kHegvMaxN) return fail(-2, "n out of range");
  if (!H) return fail(-3, "H is null");
  if (ldh < n) return fail(-4, "ldh < n");
  if (!S) return fail(-5, "S is null");
  if (lds < n) return fail(-6, "lds < n");
  if (!K) return fail(-7, "K is null");
  if (ldk < n) return fail(-8, "ldk < n");
  if (K == H || K == S) return fail(-7, "K must not alias H or S");
  if (!work) return fail(-9, "work is null");
  if (work_bytes < real_reduce_work(n)) return fail(KS_E_WORKSPACE, "workspace too small");
  if (!info_dev) return fail(-11, "info is null");
  return real_reduce_variant(variant, n, H, ldh, S, lds, K, ldk, work, info_dev, static_cast<hipStream_t>(stream));
}

int sygv_reduce_workspace_size(int32_t n, size_t* bytes) {
  if (n <= 0 || n > kHegvMaxN) return fail(-1, "n out of range");
  if (!bytes) return fail(-2, "bytes is null");
  *bytes = real_reduce_work(n);
  return 0;
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
              work, info_dev, nullptr, static_cast<hipStream_t>(stream));
}

static int check_state(const ks_plan* p, const ks_lobpcg_state* st) {
  if (!p) return fail(-1, "plan is null");
  if (!st) return fail(-3, "state is null");
  if (st->nb <= 0 || st->nb > p->nb_max) return fail(-3, "state nb out of range");
  if (st->ld < p->Ng) return fail(-3, "state ld < Ng");
  const void* ptrs[] = {st->X, st->AX, st->W, st->AW, st->P, st->AP, st->Xn, st->Pn, st->T1, st->theta, st->res,
                        st->status};
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
