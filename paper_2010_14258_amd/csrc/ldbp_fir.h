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
// LIN: no phase; out receives u and pw[j] = |u_j|^2 (summed over polarisations), the input of a
// filtered nonlinear step (nl_filter below).
// The NPOL values of one sample from LDS.  Two complex64 polarisations are read as one 16-byte access
// (a sample starts on a 16-byte boundary in every buffer): lanes RB samples apart then spread over all
// banks, where the two 8-byte accesses the compiler would otherwise emit use half of them.
template <typename R, int NPOL>
__device__ __forceinline__ void load_sample(const cx_t<R>* __restrict__ src, cx_t<R> (&v)[NPOL]) {
  if constexpr (NPOL == 2 && sizeof(R) == 4) {
    const float4 q = *reinterpret_cast<const float4*>(src);
    v[0] = float2{q.x, q.y};
    v[1] = float2{q.z, q.w};
  } else {
#pragma unroll
    for (int p = 0; p < NPOL; ++p) v[p] = src[p];
  }
}

// The NPOL values of one sample into LDS, as one 16-byte access for two complex64 polarisations.
template <typename R, int NPOL>
__device__ __forceinline__ void store_sample(cx_t<R>* __restrict__ dst, const cx_t<R> (&v)[NPOL]) {
  if constexpr (NPOL == 2 && sizeof(R) == 4) {
    *reinterpret_cast<float4*>(dst) = float4{v[0].x, v[0].y, v[1].x, v[1].y};
  } else {
#pragma unroll
    for (int p = 0; p < NPOL; ++p) dst[p] = v[p];
  }
}

template <typename R, int NPOL, int RB, int THREADS, int K, bool SYM, bool LIN = false>
__device__ __forceinline__ void fir_kerr_fixed(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out,
                                               int lo, int hi, const cx_t<R>* __restrict__ h, R coef,
                                               R* __restrict__ pw = nullptr) {
  using V = cx_t<R>;
  constexpr int W = RB + 2 * K;
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    V win[W][NPOL];
#pragma unroll
    for (int j = 0; j < W; ++j) load_sample<R, NPOL>(in + (base - K + j) * NPOL, win[j]);
    V acc[RB][NPOL];
    if constexpr (SYM) {
      const V h0 = h[K];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
          acc[r][p] = V{0, 0};
          cmac(acc[r][p], h0, win[r + K][p]);
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
      R pwr = 0;
#pragma unroll
      for (int p = 0; p < NPOL; ++p) pwr = add_power(pwr, acc[r][p]);
      if constexpr (LIN) {
        if (base + r < hi) {
          pw[base + r] = pwr;
          store_sample<R, NPOL>(out + (base + r) * NPOL, acc[r]);
        }
      } else {
        R s, co;
        phase_sincos(coef, pwr, s, co);
        if (base + r < hi) {
          V o[NPOL];
#pragma unroll
          for (int p = 0; p < NPOL; ++p) o[p] = rotate(acc[r][p], co, s);
          store_sample<R, NPOL>(out + (base + r) * NPOL, o);
        }
      }
    }
  }
}

// Filters longer than the unrolled range: taps streamed, inputs read from LDS per tap.
template <typename R, int NPOL, int RB, int THREADS, bool LIN = false>
__device__ __forceinline__ void fir_kerr_generic(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out,
                                                 int lo, int hi, int K, const cx_t<R>* __restrict__ h, R coef,
                                                 R* __restrict__ pw = nullptr) {
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
      R pwr = 0;
#pragma unroll
      for (int p = 0; p < NPOL; ++p) pwr = add_power(pwr, acc[r][p]);
      if constexpr (LIN) {
        if (base + r < hi) {
          pw[base + r] = pwr;
          store_sample<R, NPOL>(out + (base + r) * NPOL, acc[r]);
        }
      } else {
        R s, co;
        phase_sincos(coef, pwr, s, co);
        if (base + r < hi) {
          V o[NPOL];
#pragma unroll
          for (int p = 0; p < NPOL; ++p) o[p] = rotate(acc[r][p], co, s);
          store_sample<R, NPOL>(out + (base + r) * NPOL, o);
        }
      }
    }
  }
}

// KMAX: the largest half-length with a fixed-window variant compiled in (longer filters take the generic
// loop), so that a kernel instantiated for short filters does not reserve the registers of long ones.
template <typename R, int NPOL, int RB, int THREADS, bool SYM, bool LIN = false, int KMAX = 12>
__device__ __forceinline__ void fir_kerr_dispatch_t(const cx_t<R>* in, cx_t<R>* out, int lo, int hi, int K,
                                                    const cx_t<R>* h, R coef, R* pw = nullptr) {
  switch (K) {
#define LDBP_FWD_CASE(k)                                                                     \
  case k:                                                                                    \
    if constexpr (k <= KMAX) fir_kerr_fixed<R, NPOL, RB, THREADS, k, SYM, LIN>(in, out, lo, hi, h, coef, pw); \
    else fir_kerr_generic<R, NPOL, RB, THREADS, LIN>(in, out, lo, hi, K, h, coef, pw);     \
    break;
    LDBP_FWD_CASE(0) LDBP_FWD_CASE(1) LDBP_FWD_CASE(2) LDBP_FWD_CASE(3)
    LDBP_FWD_CASE(4) LDBP_FWD_CASE(5) LDBP_FWD_CASE(6) LDBP_FWD_CASE(7)
    LDBP_FWD_CASE(8) LDBP_FWD_CASE(9) LDBP_FWD_CASE(10) LDBP_FWD_CASE(11)
    LDBP_FWD_CASE(12)
#undef LDBP_FWD_CASE
    default: fir_kerr_generic<R, NPOL, RB, THREADS, LIN>(in, out, lo, hi, K, h, coef, pw); break;
  }
}

// The linear part of a filtered step: out = h * in over [lo, hi) and pw = |out|^2 there.
template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void fir_lin_dispatch(const cx_t<R>* in, cx_t<R>* out, R* pw, int lo, int hi, int K,
                                                 const cx_t<R>* h, bool sym) {
  if (sym) fir_kerr_dispatch_t<R, NPOL, RB, THREADS, true, true>(in, out, lo, hi, K, h, R(0), pw);
  else fir_kerr_dispatch_t<R, NPOL, RB, THREADS, false, true>(in, out, lo, hi, K, h, R(0), pw);
}

// Filtered nonlinear step (generalised ESSM, eq. nl_filtered with a filter per step), in place:
// u_m <- u_m exp(j coef F_m), F_m = sum_{k=-KAP}^{KAP} eta_k pw_{m-k}, for m in [lo, hi).  RB outputs
// per thread from a register window of RB + 2 KAP powers; reads pw[lo-KAP, hi+RB+KAP-2].
template <typename R, int NPOL, int RB, int THREADS, int KAP>
__device__ __forceinline__ void nl_filter_fixed(cx_t<R>* __restrict__ u, const R* __restrict__ pw, int lo, int hi,
                                                const R* __restrict__ eta, R coef) {
  using V = cx_t<R>;
  constexpr int W = RB + 2 * KAP;
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    R win[W];
#pragma unroll
    for (int j = 0; j < W; ++j) win[j] = pw[base - KAP + j];
    R F[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) F[r] = 0;
#pragma unroll
    for (int k = -KAP; k <= KAP; ++k) {
      const R e = eta[KAP + k];
#pragma unroll
      for (int r = 0; r < RB; ++r) F[r] = fma(e, win[r - k + KAP], F[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (base + r < hi) {
        R s, co;
        phase_sincos(coef, F[r], s, co);
        V a[NPOL];
        load_sample<R, NPOL>(u + (base + r) * NPOL, a);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) a[p] = rotate(a[p], co, s);
        store_sample<R, NPOL>(u + (base + r) * NPOL, a);
      }
    }
  }
}

// Runtime kappa <= KMAX with the register-window structure of nl_filter_fixed<KMAX>: the window is laid
// out for KMAX and only its entries within kappa of the outputs are loaded; taps beyond kappa are
// skipped (uniform branches), so every register index is a compile-time constant.
template <typename R, int NPOL, int RB, int THREADS, int KMAX>
__device__ __forceinline__ void nl_filter_win(cx_t<R>* __restrict__ u, const R* __restrict__ pw, int lo, int hi,
                                              int kap, const R* __restrict__ eta, R coef) {
  using V = cx_t<R>;
  constexpr int W = RB + 2 * KMAX;
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    R win[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      if (j >= KMAX - kap && j < KMAX + kap + RB) win[j] = pw[base - KMAX + j];
    }
    R F[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) F[r] = 0;
#pragma unroll
    for (int k = -KMAX; k <= KMAX; ++k) {
      if (k < -kap || k > kap) continue;
      const R e = eta[kap + k];
#pragma unroll
      for (int r = 0; r < RB; ++r) F[r] = fma(e, win[r - k + KMAX], F[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (base + r < hi) {
        R s, co;
        phase_sincos(coef, F[r], s, co);
        V a[NPOL];
        load_sample<R, NPOL>(u + (base + r) * NPOL, a);
#pragma unroll
        for (int p = 0; p < NPOL; ++p) a[p] = rotate(a[p], co, s);
        store_sample<R, NPOL>(u + (base + r) * NPOL, a);
      }
    }
  }
}

template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void nl_filter_generic(cx_t<R>* __restrict__ u, const R* __restrict__ pw, int lo, int hi,
                                                  int kap, const R* __restrict__ eta, R coef) {
  using V = cx_t<R>;
  for (int m = lo + static_cast<int>(threadIdx.x); m < hi; m += THREADS) {
    R F = 0;
    for (int k = -kap; k <= kap; ++k) F = fma(eta[kap + k], pw[m - k], F);
    R s, co;
    phase_sincos(coef, F, s, co);
    V a[NPOL];
    load_sample<R, NPOL>(u + m * NPOL, a);
#pragma unroll
    for (int p = 0; p < NPOL; ++p) a[p] = rotate(a[p], co, s);
    store_sample<R, NPOL>(u + m * NPOL, a);
  }
}

template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void nl_filter_dispatch(cx_t<R>* u, const R* pw, int lo, int hi, int kap, const R* eta,
                                                   R coef) {
  switch (kap) {
#define LDBP_NL_CASE(k) \
  case k: nl_filter_fixed<R, NPOL, RB, THREADS, k>(u, pw, lo, hi, eta, coef); break;
    LDBP_NL_CASE(0) LDBP_NL_CASE(1) LDBP_NL_CASE(2) LDBP_NL_CASE(3) LDBP_NL_CASE(4) LDBP_NL_CASE(5)
    LDBP_NL_CASE(6) LDBP_NL_CASE(8) LDBP_NL_CASE(10) LDBP_NL_CASE(12) LDBP_NL_CASE(16) LDBP_NL_CASE(20)
#undef LDBP_NL_CASE
    default:
      if (kap < 20) nl_filter_win<R, NPOL, RB, THREADS, 20>(u, pw, lo, hi, kap, eta, coef);
      else nl_filter_generic<R, NPOL, RB, THREADS>(u, pw, lo, hi, kap, eta, coef);
      break;
  }
}

template <typename R, int NPOL, int RB, int THREADS, int KMAX = 12>
__device__ __forceinline__ void fir_kerr_dispatch(const cx_t<R>* in, cx_t<R>* out, int lo, int hi, int K,
                                                  const cx_t<R>* h, R coef, bool sym = false) {
  if (sym) fir_kerr_dispatch_t<R, NPOL, RB, THREADS, true, false, KMAX>(in, out, lo, hi, K, h, coef);
  else fir_kerr_dispatch_t<R, NPOL, RB, THREADS, false, false, KMAX>(in, out, lo, hi, K, h, coef);
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
      load_sample<R, NPOL>(xw + static_cast<int64_t>(g) * NPOL, v[u]);
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int j = j0 + u * THREADS;
      if (j < W0) store_sample<R, NPOL>(buf + j * NPOL, v[u]);
    }
  }
}

// load_tile for a pass input given only on part of the circle of n samples: sample g of the pass
// input is xw[g - in_off] for 0 <= g - in_off < in_len and zero elsewhere (the zero margins of an
// aperiodic signal).  Out-of-range lanes load a clamped in-range sample and store zero, so every
// global load stays inside the in_len samples of the waveform.
template <typename R, int NPOL, int THREADS>
__device__ __forceinline__ void load_tile_edge(const cx_t<R>* __restrict__ xw, cx_t<R>* __restrict__ buf, int n,
                                               int t0, int H, int W0, int wrap_general, int in_off, int in_len) {
  using V = cx_t<R>;
  constexpr int kLoadBatch = 64 / static_cast<int>(sizeof(V) * NPOL);
  for (int j0 = threadIdx.x; j0 < W0; j0 += kLoadBatch * THREADS) {
    V v[kLoadBatch][NPOL];
    bool ok[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int j = min(j0 + u * THREADS, W0 - 1);
      int g = t0 - H + j;
      if (wrap_general) {
        g %= n;
        if (g < 0) g += n;
      } else {
        if (g < 0) g += n;
        else if (g >= n) g -= n;
      }
      const int src = g - in_off;
      ok[u] = src >= 0 && src < in_len;
      const int sc = min(max(src, 0), in_len - 1);
      load_sample<R, NPOL>(xw + static_cast<int64_t>(sc) * NPOL, v[u]);
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int j = j0 + u * THREADS;
      if (j < W0) {
        if (!ok[u]) {
#pragma unroll
          for (int p = 0; p < NPOL; ++p) v[u][p] = V{0, 0};
        }
        store_sample<R, NPOL>(buf + j * NPOL, v[u]);
      }
    }
  }
}

}  // namespace ldbp
