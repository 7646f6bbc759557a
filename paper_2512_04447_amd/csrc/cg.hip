// Training targets for the learned preconditioner: the Jacobi-Davidson
// correction equation P (H - theta_i) P t_i = P r_i, P = I - X X^H, solved by
// conjugate gradients for every column of a block at once (Sleijpen and
// van der Vorst's projected equation; Hestenes-Stiefel CG).  The literal
// (H - theta)^-1 r would return the Ritz vector itself.
//
// Each CG iteration: Ap = P (H - theta) p (H-apply, shift, projection by a
// Gram and a rotation GEMM), curvature and residual norms by deterministic
// column reductions, and per-column scalar updates.  A column stops when its
// residual falls below rtol ||P r|| or its curvature is not positive.
#include "gemm.hpp"

namespace ks {

// partial[b * nchunk + c] = Re sum_{r in chunk c} conj(a_b(r)) b_b(r)
template <typename T>
__global__ void __launch_bounds__(256)
k_coldot(const c2<T>* __restrict__ A, const c2<T>* __restrict__ B, int64_t ld, int64_t Ng, int nchunk,
         double* __restrict__ partial) {
  __shared__ double red[4];
  const int b = blockIdx.y, c = blockIdx.x;
  const int64_t per = (Ng + nchunk - 1) / nchunk;
  const int64_t r0 = (int64_t)c * per, r1 = min(Ng, r0 + per);
  const c2<T>* a = A + (int64_t)b * ld;
  const c2<T>* bb = B + (int64_t)b * ld;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const c2<T> x = a[r], y = bb[r];
    acc += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)b * nchunk + c] = acc;
}

__global__ void k_chunk_sum(const double* __restrict__ partial, int nchunk, int nb, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)b * nchunk + c];
  out[b] = s;
}

// Ap -= theta_b p
template <typename T>
__global__ void k_shift(c2<T>* __restrict__ Ap, const c2<T>* __restrict__ p, const double* __restrict__ theta, int64_t ld,
                        int64_t Ng) {
  const int b = blockIdx.y;
  const T th = (T)theta[b];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    c2<T> a = Ap[(int64_t)b * ld + r];
    const c2<T> q = p[(int64_t)b * ld + r];
    a.x -= th * q.x;
    a.y -= th * q.y;
    Ap[(int64_t)b * ld + r] = a;
  }
}

// C = -G (nb x nb, block precision) so that V + X C = V - X G.
template <typename T>
__global__ void k_proj_coef(const double2* __restrict__ G, int nb, c2<T>* __restrict__ C) {
  const int64_t total = (int64_t)nb * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double2 g = G[e];
    C[e] = cmake<c2<T>>((T)-g.x, (T)-g.y);
  }
}

// t += alpha p, res -= alpha Ap with alpha = rr / curv for active columns of
// positive curvature (0 otherwise).
template <typename T>
__global__ void k_cg_update1(c2<T>* __restrict__ t, c2<T>* __restrict__ res, const c2<T>* __restrict__ p,
                             const c2<T>* __restrict__ Ap, int64_t ld, int64_t Ng, const double* __restrict__ rr,
                             const double* __restrict__ curv, const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  const bool go = active[b] && curv[b] > 0.0;
  if (!go) return;
  const T al = (T)(rr[b] / curv[b]);
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = (int64_t)b * ld + r;
    const c2<T> q = p[i], aq = Ap[i];
    c2<T> x = t[i], s = res[i];
    x.x += al * q.x; x.y += al * q.y;
    s.x -= al * aq.x; s.y -= al * aq.y;
    t[i] = x;
    res[i] = s;
  }
}

// p = res + (rrn / rr) p for columns still active after this iteration.
template <typename T>
__global__ void k_cg_update2(c2<T>* __restrict__ p, const c2<T>* __restrict__ res, int64_t ld, int64_t Ng,
                             const double* __restrict__ rr, const double* __restrict__ rrn,
                             const double* __restrict__ curv, const double* __restrict__ bnorm, double rtol,
                             const int32_t* __restrict__ active) {
  const int b = blockIdx.y;
  if (!active[b] || !(curv[b] > 0.0) || sqrt(rrn[b]) <= rtol * bnorm[b]) return;
  const T be = (T)(rrn[b] / rr[b]);
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = (int64_t)b * ld + r;
    const c2<T> s = res[i];
    c2<T> q = p[i];
    q.x = s.x + be * q.x;
    q.y = s.y + be * q.y;
    p[i] = q;
  }
}

// Per column: stop on non-positive curvature (iters = -it) or convergence
// (iters = it); rr <- rrn.  count[0] = columns still active.
__global__ void k_cg_flags(double* __restrict__ rr, const double* __restrict__ rrn, const double* __restrict__ curv,
                           const double* __restrict__ bnorm, double rtol, int32_t* __restrict__ active,
                           int32_t* __restrict__ iters, int it, int nb, int32_t* __restrict__ count) {
  __shared__ int red[4];
  int alive = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (active[b]) {
      if (!(curv[b] > 0.0)) {
        active[b] = 0;
        iters[b] = -it;
      } else if (sqrt(rrn[b]) <= rtol * bnorm[b]) {
        active[b] = 0;
        iters[b] = it;
      } else {
        iters[b] = it;
      }
      rr[b] = rrn[b];
    }
    alive += active[b];
  }
  alive = block_sum(alive, red);
  if (threadIdx.x == 0) *count = alive;
}

__global__ void k_cg_init_flags(const double* __restrict__ rr, double* __restrict__ bnorm, int32_t* __restrict__ active,
                                int32_t* __restrict__ iters, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  bnorm[b] = sqrt(rr[b]);
  active[b] = rr[b] > 0.0 ? 1 : 0;
  iters[b] = 0;
}

// ---------------------------------------------------------------- host
struct CgWs {
  void* res;
  void* p;
  void* Ap;
  void* tmp;
  void* fft;
  void* dc;
  double2* G;
  void* C;
  double* partial;
  double* rr;
  double* rrn;
  double* curv;
  double* bnorm;
  int32_t* active;
  int32_t* count;
  void* gram;
  char* end;
};

static inline size_t al(size_t b) { return (b + 255) / 256 * 256; }
constexpr int kChunks = 64;

static CgWs cg_ws(const ks_plan& p, void* work, int nb) {
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  const size_t blk = (size_t)p.Ng * nb * es;
  char* q = static_cast<char*>(work);
  auto take = [&](size_t bytes) { char* r = q; q += al(bytes); return r; };
  CgWs w;
  w.res = take(blk);
  w.p = take(blk);
  w.Ap = take(blk);
  w.tmp = take(blk);
  w.fft = take(blk);
  w.dc = take(nl_dc_bytes(p, nb));
  w.G = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
  w.C = take((size_t)2 * nb * nb * es);
  w.partial = reinterpret_cast<double*>(take((size_t)nb * kChunks * 8));
  w.rr = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.rrn = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.curv = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.bnorm = reinterpret_cast<double*>(take((size_t)nb * 8));
  w.active = reinterpret_cast<int32_t*>(take((size_t)nb * 4));
  w.count = reinterpret_cast<int32_t*>(take(16));
  w.gram = take(gram_work_bytes(nb, p.Ng));
  w.end = q;
  return w;
}

size_t jd_work_bytes(const ks_plan& p, int nb) {
  static char probe alignas(256);
  CgWs w = cg_ws(p, &probe, nb);
  return (size_t)(w.end - &probe);
}

template <typename T>
static int coldot(const c2<T>* A, const c2<T>* B, int64_t ld, int nb, int64_t Ng, double* partial, double* out,
                  hipStream_t s) {
  hipLaunchKernelGGL((k_coldot<T>), dim3(kChunks, nb), dim3(256), 0, s, A, B, ld, Ng, kChunks, partial);
  hipLaunchKernelGGL(k_chunk_sum, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, partial, kChunks, nb, out);
  KS_LAUNCH_CHECK("coldot");
  return 0;
}

__global__ void k_sqrt_inplace(double* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = sqrt(a[i]);
}

size_t column_norms_partial(int nb) { return (size_t)nb * kChunks; }

template <typename T>
int column_norms(const c2<T>* A, int64_t ld, int nb, int64_t Ng, double* partial, double* out, hipStream_t s) {
  int rc;
  if ((rc = coldot<T>(A, A, ld, nb, Ng, partial, out, s))) return rc;
  hipLaunchKernelGGL(k_sqrt_inplace, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, out, nb);
  KS_LAUNCH_CHECK("column_norms");
  return 0;
}
template int column_norms<double>(const double2*, int64_t, int, int64_t, double*, double*, hipStream_t);
template int column_norms<float>(const float2*, int64_t, int, int64_t, double*, double*, hipStream_t);

// out = V - X (X^H V): one classical Gram-Schmidt pass (a Gram GEMM and a
// rotation GEMM).  G: nb x nb FP64 scratch; Cbuf: 2nb x nb block precision.
template <typename T>
int project_out(const c2<T>* X, const c2<T>* V, c2<T>* out, int64_t ld, int nb, int64_t Ng, double2* G, void* Cbuf,
                void* gram_ws, hipStream_t s) {
  int rc;
  BlockList<c2<T>> LX{{X, nullptr, nullptr}, ld, nb};
  BlockList<c2<T>> LV{{V, nullptr, nullptr}, ld, nb};
  if ((rc = gram_general<T>(LX, LV, nb, Ng, G, nb, gram_ws, s))) return rc;
  hipLaunchKernelGGL((k_proj_coef<T>), dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)nb * nb, 256), 4096)),
                     dim3(256), 0, s, G, nb, static_cast<c2<T>*>(Cbuf));
  KS_LAUNCH_CHECK("proj_coef");
  // out = V + X (-X^H V): the first nb rows of the coefficients, V added in
  // the rotation's epilogue
  return rotate<T>(LX, nb, nb, static_cast<const c2<T>*>(Cbuf), nb, nb, Ng, out, nullptr, ld, s, false, V);
}

template int project_out<double>(const double2*, const double2*, double2*, int64_t, int, int64_t, double2*, void*,
                                 void*, hipStream_t);
template int project_out<float>(const float2*, const float2*, float2*, int64_t, int, int64_t, double2*, void*, void*,
                                hipStream_t);

template <typename T>
static int project(const ks_plan& p, const CgWs& w, const c2<T>* X, const c2<T>* V, c2<T>* out, int64_t ld, int nb,
                   hipStream_t s) {
  return project_out<T>(X, V, out, ld, nb, p.Ng, w.G, w.C, w.gram, s);
}

template <typename T>
int jd_correction(const ks_plan& p, const T* v, const c2<T>* X, const double* theta, const c2<T>* R, int64_t ld,
                  int nb, int maxit, double rtol, c2<T>* Tout, int32_t* iters, void* work, hipStream_t s) {
  using T2 = c2<T>;
  CgWs w = cg_ws(p, work, nb);
  int rc;
  T2* res = static_cast<T2*>(w.res);
  T2* pv = static_cast<T2*>(w.p);
  T2* Ap = static_cast<T2*>(w.Ap);
  T2* tmp = static_cast<T2*>(w.tmp);
  const dim3 eg((unsigned)std::min<int64_t>(ceil_div(p.Ng, 256), 256), nb);
  // b = P r; res = p = b; t = 0
  if ((rc = project<T>(p, w, X, R, res, ld, nb, s))) return rc;
  KS_HIP(hipMemcpy2DAsync(pv, ld * sizeof(T2), res, ld * sizeof(T2), p.Ng * sizeof(T2), nb, hipMemcpyDeviceToDevice, s));
  KS_HIP(hipMemset2DAsync(Tout, ld * sizeof(T2), 0, p.Ng * sizeof(T2), nb, s));
  if ((rc = coldot<T>(res, res, ld, nb, p.Ng, w.partial, w.rr, s))) return rc;
  hipLaunchKernelGGL(k_cg_init_flags, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, s, w.rr, w.bnorm, w.active,
                     iters, nb);
  KS_LAUNCH_CHECK("cg_init");
  for (int it = 1; it <= maxit; ++it) {
    if ((rc = apply_h<T>(p, v, pv, ld, Ap, ld, nb, static_cast<T2*>(w.fft), static_cast<T2*>(w.dc), s))) return rc;
    hipLaunchKernelGGL((k_shift<T>), eg, dim3(256), 0, s, Ap, pv, theta, ld, p.Ng);
    KS_LAUNCH_CHECK("shift");
    if ((rc = project<T>(p, w, X, Ap, tmp, ld, nb, s))) return rc;
    if ((rc = coldot<T>(pv, tmp, ld, nb, p.Ng, w.partial, w.curv, s))) return rc;
    hipLaunchKernelGGL((k_cg_update1<T>), eg, dim3(256), 0, s, Tout, res, pv, tmp, ld, p.Ng, w.rr, w.curv, w.active);
    KS_LAUNCH_CHECK("cg_update1");
    if ((rc = coldot<T>(res, res, ld, nb, p.Ng, w.partial, w.rrn, s))) return rc;
    hipLaunchKernelGGL((k_cg_update2<T>), eg, dim3(256), 0, s, pv, res, ld, p.Ng, w.rr, w.rrn, w.curv, w.bnorm, rtol,
                       w.active);
    KS_LAUNCH_CHECK("cg_update2");
    hipLaunchKernelGGL(k_cg_flags, dim3(1), dim3(256), 0, s, w.rr, w.rrn, w.curv, w.bnorm, rtol, w.active, iters, it,
                       nb, w.count);
    KS_LAUNCH_CHECK("cg_flags");
    if (it % 16 == 0 || it == maxit) {
      int32_t alive = 0;
      KS_HIP(hipMemcpyAsync(&alive, w.count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      KS_HIP(hipStreamSynchronize(s));
      if (alive == 0) break;
    }
  }
  // final projection t <- P t
  if ((rc = project<T>(p, w, X, Tout, tmp, ld, nb, s))) return rc;
  KS_HIP(hipMemcpy2DAsync(Tout, ld * sizeof(T2), tmp, ld * sizeof(T2), p.Ng * sizeof(T2), nb, hipMemcpyDeviceToDevice, s));
  return 0;
}

template int jd_correction<double>(const ks_plan&, const double*, const double2*, const double*, const double2*, int64_t,
                                   int, int, double, double2*, int32_t*, void*, hipStream_t);
template int jd_correction<float>(const ks_plan&, const float*, const float2*, const double*, const float2*, int64_t,
                                  int, int, double, float2*, int32_t*, void*, hipStream_t);

}  // namespace ks
