// Shared device/host helpers of the LDBP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ldbp.h"

namespace ldbp {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int status, const char* fmt, ...);

#define LDBP_HIP_CHECK(expr)                                                         \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::ldbp::fail(LDBP_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- complex types
template <typename R> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };
template <typename R> using cx_t = typename cx<R>::type;

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// acc += h * v (4 fused multiply-adds)
template <typename V>
__device__ __forceinline__ void cmac(V& acc, V h, V v) {
  acc.x = fma(h.x, v.x, acc.x);
  acc.x = fma(-h.y, v.y, acc.x);
  acc.y = fma(h.x, v.y, acc.y);
  acc.y = fma(h.y, v.x, acc.y);
}

// acc += conj(h) * v
template <typename V>
__device__ __forceinline__ void cmac_conj(V& acc, V h, V v) {
  acc.x = fma(h.x, v.x, acc.x);
  acc.x = fma(h.y, v.y, acc.x);
  acc.y = fma(h.x, v.y, acc.y);
  acc.y = fma(-h.y, v.x, acc.y);
}

// Kerr phase rotation helpers.  For float the hardware sine/cosine (input in
// revolutions) is used after reducing the argument to [-1/2, 1/2] revolutions;
// the caller passes the coefficient already divided by 2*pi.  For double the
// library sincos is called with the phase in radians.
struct Rot32 {
  __device__ __forceinline__ static void sincos_rev(float rev, float& s, float& c) {
    rev = rev - __builtin_rintf(rev);
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
  }
};

// The fused reduction: the exact product minus the integer nearest its rounded value, in one operation.
__device__ __forceinline__ void phase_sincos(float coef_rev, float p, float& s, float& c) {
  const float rev = fmaf(coef_rev, p, -__builtin_rintf(coef_rev * p));
  s = __builtin_amdgcn_sinf(rev);
  c = __builtin_amdgcn_cosf(rev);
}
__device__ __forceinline__ void phase_sincos(double coef_rad, double p, double& s, double& c) {
  sincos(coef_rad * p, &s, &c);
}

// |v|^2 added to p, and v (c + j s), with every product fused explicitly.  The forward's arithmetic is
// written without an unfused multiply feeding an add, so that the compiler has no contraction left to
// choose: each inlined and unrolled copy then rounds alike, and an output does not depend on where the
// tiling puts it in a thread's register window.
template <typename V, typename R>
__device__ __forceinline__ R add_power(R p, const V& v) {
  return fma(v.y, v.y, fma(v.x, v.x, p));
}
template <typename V, typename R>
__device__ __forceinline__ V rotate(const V& v, R c, R s) {
  return V{fma(v.x, c, -(v.y * s)), fma(v.x, s, v.y * c)};
}

// Coefficient as the kernels consume it: revolutions for float, radians for double.
template <typename R> __host__ __device__ inline R phase_coef_scale();
template <> __host__ __device__ inline float phase_coef_scale<float>() { return 0.15915494309189535f; }
template <> __host__ __device__ inline double phase_coef_scale<double>() { return 1.0; }

inline size_t real_size(int dtype) { return dtype == LDBP_C64 ? sizeof(float) : sizeof(double); }
inline size_t cx_size(int dtype) { return 2 * real_size(dtype); }

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace ldbp
