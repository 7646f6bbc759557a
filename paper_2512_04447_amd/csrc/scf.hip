// The self-consistent loop's steps around the eigensolve (the "Others" of
// the paper's SCF cost breakdown): electron density from the occupied
// orbitals, the Hartree potential by the periodic Poisson equation on the
// FFT passes, a local density approximation for exchange and correlation
// (Slater exchange, Perdew-Zunger correlation), the effective potential with
// its grid sums, and linear density mixing.  Every reduction sums partials
// in a fixed order.
#include <cmath>

#include "gemm.hpp"

namespace ks {

constexpr int kScfThreads = 256;
constexpr int kScfBlocks = 1024;  // partial sums per reduction

// n(r) = sum_i f_i |x_i(r)|^2, one thread per grid point; bands in groups
// of eight loads in flight.
template <typename T>
__global__ void __launch_bounds__(kScfThreads)
k_density(const c2<T>* __restrict__ X, int64_t ld, int nocc, const double* __restrict__ occ, int64_t Ng,
          double* __restrict__ n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i0 = 0; i0 < nocc; i0 += 8) {
      c2<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = X[(int64_t)min(i0 + u, nocc - 1) * ld + r];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double f = i0 + u < nocc ? (occ ? occ[i0 + u] : 2.0) : 0.0;
        acc += f * ((double)v[u].x * v[u].x + (double)v[u].y * v[u].y);
      }
    }
    n[r] = acc;
  }
}

// Slater exchange and Perdew-Zunger correlation for the density per volume
// rho (Perdew and Zunger, Phys. Rev. B 23, 5048 (1981)); rho <= 1e-30 gives 0.
__device__ inline void lda_point(double rho, double& exc, double& vxc) {
  if (!(rho > 1e-30)) {
    exc = 0.0;
    vxc = 0.0;
    return;
  }
  const double ex = -0.75 * cbrt(3.0 * rho / M_PI);
  const double rs = cbrt(3.0 / (4.0 * M_PI * rho));
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double lr = log(rs);
    ec = A * lr + B + C * rs * lr + D * rs;
    vc = A * lr + (B - A / 3.0) + 2.0 / 3.0 * C * rs * lr + (2.0 * D - C) / 3.0 * rs;
  }
  exc = ex + ec;
  vxc = 4.0 / 3.0 * ex + vc;
}

__global__ void __launch_bounds__(kScfThreads)
k_lda(const double* __restrict__ n, double inv_dv, int64_t Ng, double* __restrict__ vxc, double* __restrict__ exc) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    double e, v;
    lda_point(n[r] * inv_dv, e, v);
    vxc[r] = v;
    if (exc) exc[r] = e;
  }
}

// complex field rho = n / dV (imaginary part 0); slot `one` set to 1.
template <typename T>
__global__ void k_rho_field(const double* __restrict__ n, double inv_dv, int64_t Ng, c2<T>* __restrict__ f,
                            double* __restrict__ one) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *one = 1.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x)
    f[r] = cmake<c2<T>>((T)(n[r] * inv_dv), T(0));
}

template <typename T>
__global__ void k_real_part(const c2<T>* __restrict__ f, int64_t Ng, double* __restrict__ v) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x)
    v[r] = (double)f[r].x;
}

__device__ inline double block_sum_scf(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x / 64); ++i) t += red[i];
  return t;
}

// V_eff = V_ion + V_H + v_xc in the plan precision, and per-block partial
// sums of V_H n, v_xc n, e_xc n and n.
template <typename T>
__global__ void __launch_bounds__(kScfThreads)
k_combine(const double* __restrict__ n, const double* __restrict__ v_ion, const double* __restrict__ vh,
          const double* __restrict__ vxc, const double* __restrict__ exc, int64_t Ng, T* __restrict__ v_eff,
          double* __restrict__ partial) {
  __shared__ double red[kScfThreads / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    const double nr = n[r], h = vh[r], x = vxc[r];
    v_eff[r] = (T)(v_ion[r] + h + x);
    s0 += h * nr;
    s1 += x * nr;
    s2 += exc[r] * nr;
    s3 += nr;
  }
  const double t0 = block_sum_scf(s0, red), t1 = block_sum_scf(s1, red), t2 = block_sum_scf(s2, red),
               t3 = block_sum_scf(s3, red);
  if (threadIdx.x == 0) {
    partial[4 * blockIdx.x + 0] = t0;
    partial[4 * blockIdx.x + 1] = t1;
    partial[4 * blockIdx.x + 2] = t2;
    partial[4 * blockIdx.x + 3] = t3;
  }
}

// out[k] = sum over blocks (ascending) of partial[w * b + k], k < w
__global__ void k_sum_partials(const double* __restrict__ partial, int nblk, int w, double* __restrict__ out) {
  if (threadIdx.x < w) {
    double t = 0.0;
    for (int b2 = 0; b2 < nblk; ++b2) t += partial[w * b2 + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kScfThreads)
k_mix(double alpha, const double* __restrict__ n_in, const double* __restrict__ n_out, int64_t Ng,
      double* __restrict__ n_next, double* __restrict__ partial) {
  __shared__ double red[kScfThreads / 64];
  double s = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < Ng; r += (int64_t)gridDim.x * blockDim.x) {
    const double a = n_in[r], o = n_out[r];
    n_next[r] = (1.0 - alpha) * a + alpha * o;
    s += (o - a) * (o - a);
  }
  const double t = block_sum_scf(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_sqrt_sum(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b2 = 0; b2 < nblk; ++b2) t += partial[b2];
    *out = sqrt(t);
  }
}

static unsigned scf_grid(int64_t Ng) { return (unsigned)std::min<int64_t>(ceil_div(Ng, kScfThreads), kScfBlocks); }

struct ScfWs {
  void* f0;  // complex Ng, plan precision
  void* f1;
  double* vh;
  double* vxc;
  double* exc;
  double* partial;  // 4 kScfBlocks
  double* one;
  char* end;
};

static ScfWs scf_ws(const ks_plan& p, void* work) {
  const size_t es = p.prec == KS_FP64 ? 16 : 8;
  char* q = static_cast<char*>(work);
  auto take = [&](size_t bytes) { char* r = q; q += (bytes + 255) / 256 * 256; return r; };
  ScfWs w;
  w.f0 = take((size_t)p.Ng * es);
  w.f1 = take((size_t)p.Ng * es);
  w.vh = reinterpret_cast<double*>(take((size_t)p.Ng * 8));
  w.vxc = reinterpret_cast<double*>(take((size_t)p.Ng * 8));
  w.exc = reinterpret_cast<double*>(take((size_t)p.Ng * 8));
  w.partial = reinterpret_cast<double*>(take((size_t)4 * kScfBlocks * 8));
  w.one = reinterpret_cast<double*>(take(8));
  w.end = q;
  return w;
}

size_t scf_work_bytes(const ks_plan& p) {
  static char probe alignas(256);
  return (size_t)(scf_ws(p, &probe).end - &probe);
}

int density_impl(const ks_plan& p, const void* X, int64_t ld, int nocc, const double* occ, double* n, hipStream_t s) {
  if (p.prec == KS_FP64)
    hipLaunchKernelGGL((k_density<double>), dim3(scf_grid(p.Ng)), dim3(kScfThreads), 0, s,
                       static_cast<const double2*>(X), ld, nocc, occ, p.Ng, n);
  else
    hipLaunchKernelGGL((k_density<float>), dim3(scf_grid(p.Ng)), dim3(kScfThreads), 0, s,
                       static_cast<const float2*>(X), ld, nocc, occ, p.Ng, n);
  KS_LAUNCH_CHECK("density");
  return 0;
}

static double grid_dv(const ks_plan& p) {
  return p.grid.L[0] * p.grid.L[1] * p.grid.L[2] / (double)p.Ng;
}

template <typename T>
static int hartree_t(const ks_plan& p, const double* n, double* vh, const ScfWs& w, hipStream_t s) {
  auto* f0 = static_cast<c2<T>*>(w.f0);
  auto* f1 = static_cast<c2<T>*>(w.f1);
  hipLaunchKernelGGL((k_rho_field<T>), dim3(scf_grid(p.Ng)), dim3(kScfThreads), 0, s, n, 1.0 / grid_dv(p), p.Ng,
                     f0, w.one);
  int rc;
  if ((rc = poisson<T>(p, f0, f1, f0, w.one, s))) return rc;
  hipLaunchKernelGGL((k_real_part<T>), dim3(scf_grid(p.Ng)), dim3(kScfThreads), 0, s, f0, p.Ng, vh);
  KS_LAUNCH_CHECK("hartree");
  return 0;
}

int hartree_impl(const ks_plan& p, const double* n, double* vh, void* work, hipStream_t s) {
  const ScfWs w = scf_ws(p, work);
  return p.prec == KS_FP64 ? hartree_t<double>(p, n, vh, w, s) : hartree_t<float>(p, n, vh, w, s);
}

int lda_impl(const ks_plan& p, const double* n, double* vxc, double* exc, hipStream_t s) {
  hipLaunchKernelGGL(k_lda, dim3(scf_grid(p.Ng)), dim3(kScfThreads), 0, s, n, 1.0 / grid_dv(p), p.Ng, vxc, exc);
  KS_LAUNCH_CHECK("lda");
  return 0;
}

int scf_potential_impl(const ks_plan& p, const double* n, const double* v_ion, void* v_eff, double* terms,
                       void* work, hipStream_t s) {
  const ScfWs w = scf_ws(p, work);
  int rc;
  if ((rc = hartree_impl(p, n, w.vh, work, s))) return rc;
  if ((rc = lda_impl(p, n, w.vxc, w.exc, s))) return rc;
  const unsigned g = scf_grid(p.Ng);
  if (p.prec == KS_FP64)
    hipLaunchKernelGGL((k_combine<double>), dim3(g), dim3(kScfThreads), 0, s, n, v_ion, w.vh, w.vxc, w.exc, p.Ng,
                       static_cast<double*>(v_eff), w.partial);
  else
    hipLaunchKernelGGL((k_combine<float>), dim3(g), dim3(kScfThreads), 0, s, n, v_ion, w.vh, w.vxc, w.exc, p.Ng,
                       static_cast<float*>(v_eff), w.partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, w.partial, (int)g, 4, terms);
  KS_LAUNCH_CHECK("scf_potential");
  return 0;
}

int mix_impl(const ks_plan& p, double alpha, const double* n_in, const double* n_out, double* n_next, double* resid,
             void* work, hipStream_t s) {
  const ScfWs w = scf_ws(p, work);
  const unsigned g = scf_grid(p.Ng);
  hipLaunchKernelGGL(k_mix, dim3(g), dim3(kScfThreads), 0, s, alpha, n_in, n_out, p.Ng, n_next, w.partial);
  hipLaunchKernelGGL(k_sqrt_sum, dim3(1), dim3(64), 0, s, w.partial, (int)g, resid);
  KS_LAUNCH_CHECK("mix");
  return 0;
}

}  // namespace ks
