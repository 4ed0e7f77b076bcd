// Device operations of a split-step program shared by its kernels (ssm.hip, ssm_var.hip): the
// pointwise operation between linear steps and the linear step's response on the DFT grid
// (Sec. III-A, eq. discretized_nlse; Sec. IV-A for the amplifier gain and noise).
#pragma once

#include "common.h"

namespace ldbp {

// Pointwise operation of the program, as the kernels consume it.
struct PwOp {
  double ka, g, sigma, kb;
  int32_t slot;  // noise slot or -1
  int32_t pad;
};

// Per-sample Kerr phase for a time sample of NPOL complex values held at v[0..NPOL).
template <typename R>
__device__ __forceinline__ void kerr_rotate(cx_t<R>* v, int npol, double k) {
  if (k == 0.0) return;
  R p = 0;
  for (int q = 0; q < npol; ++q) p += v[q].x * v[q].x + v[q].y * v[q].y;
  R s, c;
  phase_sincos(static_cast<R>(k) * phase_coef_scale<R>(), p, s, c);
  for (int q = 0; q < npol; ++q) {
    const cx_t<R> o = v[q];
    v[q] = cx_t<R>{o.x * c - o.y * s, o.x * s + o.y * c};
  }
}

template <typename R>
__device__ __forceinline__ void apply_pw(cx_t<R>* v, int npol, const PwOp& op, const cx_t<R>* noise_at) {
  kerr_rotate<R>(v, npol, op.ka);
  if (op.g != 1.0) {
    const R g = static_cast<R>(op.g);
    for (int q = 0; q < npol; ++q) v[q] = cx_t<R>{v[q].x * g, v[q].y * g};
  }
  if (noise_at) {
    const R s = static_cast<R>(op.sigma);
    for (int q = 0; q < npol; ++q) v[q] = cx_t<R>{v[q].x + s * noise_at[q].x, v[q].y + s * noise_at[q].y};
  }
  kerr_rotate<R>(v, npol, op.kb);
}

// exp(z (j beta2 w^2/2 - alpha/2)) / n for FFT bin k of an n-point grid at rate fs.
template <typename R>
__device__ __forceinline__ cx_t<R> lin_response(int64_t k, int64_t n, double zrev, R amp) {
  // zrev = z beta2 pi fs^2 / n^2: the phase in revolutions is zrev * m^2, m the signed bin index
  const double m = static_cast<double>(k < (n + 1) / 2 ? k : k - n);
  double rev = zrev * m * m;
  rev -= rint(rev);
  R s, c;
  if constexpr (sizeof(R) == 4) {
    Rot32::sincos_rev(static_cast<float>(rev), s, c);
  } else {
    sincos(6.283185307179586476925 * rev, &s, &c);
  }
  return cx_t<R>{amp * c, amp * s};
}

}  // namespace ldbp
