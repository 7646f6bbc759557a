// Shared device/host helpers of the ksh library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ksh.h"

namespace ks {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define KS_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::ks::hip_fail(e_, #call); \
  } while (0)

#define KS_LAUNCH_CHECK(what)                          \
  do {                                                 \
    hipError_t e_ = hipGetLastError();                 \
    if (e_ != hipSuccess) return ::ks::hip_fail(e_, what); \
  } while (0)

// ------------------------------------------------------------------ timing
// Event pair around launches of one kernel family when enabled (see
// ks_kernel_timer in ksh.h); no-ops otherwise.
enum KernelFamily {
  KF_GRAM = 0, KF_ROTATE, KF_PASS_A, KF_PASS_B, KF_PASS_C, KF_NL_PROJECT, KF_HEGV, KF_ZGEMM, KF_GRAM_BASIS,
  KF_NL_SCATTER
};
void timer_begin(int family, hipStream_t s);
void timer_end(int family, hipStream_t s);

struct TimerScope {
  int f;
  hipStream_t s;
  TimerScope(int family, hipStream_t st) : f(family), s(st) { timer_begin(f, s); }
  ~TimerScope() { timer_end(f, s); }
};

// ------------------------------------------------------------------ complex
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using c2 = typename cvec<T>::type;

template <typename T2> __device__ __host__ inline T2 cmake(decltype(T2{}.x) re, decltype(T2{}.x) im) {
  T2 r; r.x = re; r.y = im; return r;
}
template <typename T2> __device__ __host__ inline T2 cadd(T2 a, T2 b) { a.x += b.x; a.y += b.y; return a; }
template <typename T2> __device__ __host__ inline T2 csub(T2 a, T2 b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename T2> __device__ __host__ inline T2 cmul(T2 a, T2 b) {
  T2 r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename T2> __device__ __host__ inline T2 cmulc(T2 a, T2 b) {
  T2 r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename T2> __device__ __host__ inline T2 cconj(T2 a) { a.y = -a.y; return a; }
template <typename T2, typename S> __device__ __host__ inline T2 cscale(T2 a, S s) { a.x *= s; a.y *= s; return a; }
template <typename T2> __device__ __host__ inline decltype(T2{}.x) cabs2(T2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ loads
// Load through a global (address space 1) pointer.  Where the compiler
// cannot prove that a generic pointer is global (pointers read from a
// struct, or selected against null) it emits flat loads, which count on
// the LDS wait counter as well: every LDS read after them then waits for
// the global load to return, and a register prefetch no longer overlaps
// the arithmetic.  The pointer must address device global memory.
// (Loaded as a clang vector type: the HIP vector structs have no copy from
// an address-space-qualified object.)
__device__ __forceinline__ double2 gload(const double2* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gload(const float2* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return make_float2(v.x, v.y);
}

// ------------------------------------------------------------------ launch order
// The device deals consecutive workgroups of a launch to its eight XCDs in
// turn, each XCD with its own L2.  xcd_order renumbers workgroup g of G so
// that the workgroups one XCD receives form one contiguous range of the
// new index (a bijection of [0, G)): workgroups that share input then run
// on the same XCD at about the same time and meet it in its L2.
__device__ __forceinline__ int64_t xcd_order(int64_t g, int64_t G) {
  const int64_t per = G / 8, rem = G % 8, x = g % 8;
  return x * per + (x < rem ? x : rem) + g / 8;
}

// ------------------------------------------------------------------ reductions
constexpr int kWave = 64;

template <typename T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Deterministic block sum (fixed tree); every thread gets the result.
// `red` must hold blockDim.x/64 elements.  Ends with a barrier.
template <typename T> __device__ inline T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = T(0);
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace ks
