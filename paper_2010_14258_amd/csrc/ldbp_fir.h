// Device building blocks shared by the LDBP forward and backward kernels:
// register-blocked circular FIR + Kerr phase over an LDS-resident signal.
#pragma once

#include "common.h"

namespace ldbp {

// out[j] = sigma(sum_{k=-K}^{K} h_k in[j-k]) for j in [lo, hi), RB consecutive outputs per thread
// from a register window of RB + 2K inputs.  Reads in[lo-K, hi+RB+K-2]; writes out[lo, hi).
// SYM: the caller guarantees h_{-k} = h_k and the sum is evaluated folded,
// h_0 x_m + sum_{k>=1} h_k (x_{m-k} + x_{m+k}) (the folded structure of Sec. III-B), which
// needs K + 1 complex multiplies instead of 2K + 1.
// An odd RB keeps the lanes' window starts on distinct LDS banks (stride RB * 8 bytes).
template <typename R, int NPOL, int RB, int THREADS, int K, bool SYM>
__device__ __forceinline__ void fir_kerr_fixed(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out,
                                               int lo, int hi, const cx_t<R>* __restrict__ h, R coef) {
  using V = cx_t<R>;
  constexpr int W = RB + 2 * K;
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    V win[W][NPOL];
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int p = 0; p < NPOL; ++p) win[j][p] = in[(base - K + j) * NPOL + p];
    V acc[RB][NPOL];
    if constexpr (SYM) {
      const V h0 = h[K];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
          const V c = win[r + K][p];
          acc[r][p] = V{h0.x * c.x - h0.y * c.y, h0.x * c.y + h0.y * c.x};
        }
#pragma unroll
      for (int k = 1; k <= K; ++k) {
        const V hk = h[K + k];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int p = 0; p < NPOL; ++p) {
            const V a = win[r + K - k][p], b = win[r + K + k][p];
            cmac(acc[r][p], hk, V{a.x + b.x, a.y + b.y});
          }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int p = 0; p < NPOL; ++p) acc[r][p] = V{0, 0};
#pragma unroll
      for (int k = -K; k <= K; ++k) {
        const V hk = h[K + k];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int p = 0; p < NPOL; ++p) cmac(acc[r][p], hk, win[r - k + K][p]);  // x_{m-k}, m = base + r
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      R pw = 0;
#pragma unroll
      for (int p = 0; p < NPOL; ++p) pw += acc[r][p].x * acc[r][p].x + acc[r][p].y * acc[r][p].y;
      R s, co;
      phase_sincos(coef, pw, s, co);
      if (base + r < hi) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
          V o;
          o.x = acc[r][p].x * co - acc[r][p].y * s;
          o.y = acc[r][p].x * s + acc[r][p].y * co;
          out[(base + r) * NPOL + p] = o;
        }
      }
    }
  }
}

// Filters longer than the unrolled range: taps streamed, inputs read from LDS per tap.
template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void fir_kerr_generic(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out,
                                                 int lo, int hi, int K, const cx_t<R>* __restrict__ h, R coef) {
  using V = cx_t<R>;
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    V acc[RB][NPOL];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int p = 0; p < NPOL; ++p) acc[r][p] = V{0, 0};
    for (int k = -K; k <= K; ++k) {
      const V hk = h[K + k];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int p = 0; p < NPOL; ++p) cmac(acc[r][p], hk, in[(base + r - k) * NPOL + p]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      R pw = 0;
#pragma unroll
      for (int p = 0; p < NPOL; ++p) pw += acc[r][p].x * acc[r][p].x + acc[r][p].y * acc[r][p].y;
      R s, co;
      phase_sincos(coef, pw, s, co);
      if (base + r < hi) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
          V o;
          o.x = acc[r][p].x * co - acc[r][p].y * s;
          o.y = acc[r][p].x * s + acc[r][p].y * co;
          out[(base + r) * NPOL + p] = o;
        }
      }
    }
  }
}

template <typename R, int NPOL, int RB, int THREADS, bool SYM>
__device__ __forceinline__ void fir_kerr_dispatch_t(const cx_t<R>* in, cx_t<R>* out, int lo, int hi, int K,
                                                    const cx_t<R>* h, R coef) {
  switch (K) {
#define LDBP_FWD_CASE(k) \
  case k: fir_kerr_fixed<R, NPOL, RB, THREADS, k, SYM>(in, out, lo, hi, h, coef); break;
    LDBP_FWD_CASE(0) LDBP_FWD_CASE(1) LDBP_FWD_CASE(2) LDBP_FWD_CASE(3)
    LDBP_FWD_CASE(4) LDBP_FWD_CASE(5) LDBP_FWD_CASE(6) LDBP_FWD_CASE(7)
    LDBP_FWD_CASE(8) LDBP_FWD_CASE(9) LDBP_FWD_CASE(10) LDBP_FWD_CASE(11)
    LDBP_FWD_CASE(12)
#undef LDBP_FWD_CASE
    default: fir_kerr_generic<R, NPOL, RB, THREADS>(in, out, lo, hi, K, h, coef); break;
  }
}

template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void fir_kerr_dispatch(const cx_t<R>* in, cx_t<R>* out, int lo, int hi, int K,
                                                  const cx_t<R>* h, R coef, bool sym = false) {
  if (sym) fir_kerr_dispatch_t<R, NPOL, RB, THREADS, true>(in, out, lo, hi, K, h, coef);
  else fir_kerr_dispatch_t<R, NPOL, RB, THREADS, false>(in, out, lo, hi, K, h, coef);
}

// Loads samples [t0 - H, t0 + Lw + H) of one waveform (circularly) into LDS.  Each thread issues a
// batch of global loads (64 bytes of samples) before its first LDS store, so the loads of a tile are
// in flight together instead of one round trip per element.
template <typename R, int NPOL, int THREADS>
__device__ __forceinline__ void load_tile(const cx_t<R>* __restrict__ xw, cx_t<R>* __restrict__ buf, int n,
                                          int t0, int H, int W0, int wrap_general) {
  using V = cx_t<R>;
  constexpr int kLoadBatch = 64 / static_cast<int>(sizeof(V) * NPOL);
  for (int j0 = threadIdx.x; j0 < W0; j0 += kLoadBatch * THREADS) {
    V v[kLoadBatch][NPOL];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int j = min(j0 + u * THREADS, W0 - 1);  // past the end: reload the last sample, not stored
      int g = t0 - H + j;
      if (wrap_general) {
        g %= n;
        if (g < 0) g += n;
      } else {
        if (g < 0) g += n;
        else if (g >= n) g -= n;
      }
#pragma unroll
      for (int p = 0; p < NPOL; ++p) v[u][p] = xw[static_cast<int64_t>(g) * NPOL + p];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int j = j0 + u * THREADS;
      if (j < W0)
#pragma unroll
        for (int p = 0; p < NPOL; ++p) buf[j * NPOL + p] = v[u][p];
    }
  }
}

}  // namespace ldbp
