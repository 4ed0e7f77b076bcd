// LDBP backward: adjoint of the time-blocked forward, recomputing from block checkpoints.
//
// The model (eq. model, Sec. III-B) is differentiated step by step; the paper
// trains with standard tools, so this adjoint is the chain rule written out:
//   Kerr  y = u e^{j phi}, phi = c P(u), P = |u|^2 (summed over polarisations):
//         q = Im(G_y conj(y)),  dc += q P,  G_u = (G_y + 2 c q y) e^{-j phi}
//         (using u = y e^{-j phi} and P(u) = P(y), so only y is kept)
//   FIR   u_m = sum_k h_k x_{m-k}:
//         dh_k += G_u,m conj(x_{m-k}),  G_x,p = sum_k conj(h_k) G_u,(p+k)
// with G = dL/dRe + j dL/dIm.
//
// One workgroup handles a tile of L block-input positions [t0, t0+L) of one
// block of S steps (halo H = sum K):
//   1. load the block input over [t0-2H, t0+L+2H) and recompute y_1..y_S in LDS,
//      y_s kept over [t0-(2H-h_s), t0+L+(2H-h_s)), h_s = K_1 + ... + K_s;
//   2. load the block-output gradient over [t0-H, t0+L+H);
//   3. for s = S..1: Kerr adjoint over [t0-h_s, t0+L+h_s), FIR adjoint down to
//      [t0-h_{s-1}, t0+L+h_{s-1}), tap and Kerr-coefficient gradients summed over
//      the tile's own positions only (each position is owned by one tile; the tap
//      correlation of filters up to 25 taps is taken in the FIR adjoint's pass as
//      sum_{owned p} G_u,(p+k) conj(x_p));
//   4. write the block-input gradient over [t0, t0+L) and the tile's partial
//      sums (one FP64 value per tap and step) to a [tile][column] buffer that a
//      second kernel reduces in a fixed order, so results are deterministic.
// Symmetric filters (h_{-k} = h_k) are evaluated folded in all three FIR products:
//   recompute  u_m = h_0 x_m + sum_{k>=1} h_k (x_{m-k} + x_{m+k})
//   adjoint    G_x,p = conj(h_0) G_u,p + sum_{k>=1} conj(h_k) (G_u,(p+k) + G_u,(p-k))
//   taps       g_k = sum_m G_u,m conj(x_{m-k} + x_{m+k}) = dL/dh_k + dL/dh_{-k}  (k >= 1)
// and the tap gradient is returned as its projection on symmetric filters, g_k / 2 in both
// entries k and -k (g_0 = dL/dh_0 in the centre).
#include <algorithm>
#include <vector>

#include "common.h"
#include "ldbp_fir.h"
#include "ldbp_kernels.h"

namespace ldbp {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DPP source operand: the value of another lane selected by `ctrl` (0 where masked or out of range).
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                                               BANK_MASK, true));
}

// Sum over the 64 lanes of a wave using row shifts and row broadcasts (full-rate VALU adds, no
// LDS round trip); the total is valid in lane 63 only.
__device__ __forceinline__ float wave_sum_last(float v) {
  float s = v + dpp_f32<0x111, 0xf, 0xf>(v);    // row_shr:1
  s += dpp_f32<0x112, 0xf, 0xf>(v);             // row_shr:2
  s += dpp_f32<0x113, 0xf, 0xf>(v);             // row_shr:3   -> lane i holds v[i-3..i] within its row
  s += dpp_f32<0x114, 0xf, 0xe>(s);             // row_shr:4, banks 1-3 -> 8-lane partial sums
  s += dpp_f32<0x118, 0xf, 0xc>(s);             // row_shr:8, banks 2-3 -> lane 15 of a row holds the row sum
  s += dpp_f32<0x142, 0xa, 0xf>(s);             // row_bcast:15 into rows 1, 3
  s += dpp_f32<0x143, 0xc, 0xf>(s);             // row_bcast:31 into rows 2, 3 -> lane 63 holds the total
  return s;
}
__device__ __forceinline__ double wave_sum_last(double v) { return wave_sum(v); }

constexpr int kLastLane = 63;

// Value of the lane whose index differs in bit B (within a row of 16 lanes, B < 4).
template <int B>
__device__ __forceinline__ float lane_xor(float v) {
  const int x = __builtin_bit_cast(int, v);
  int r;
  if constexpr (B == 0) {
    r = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
  } else if constexpr (B == 1) {
    r = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
  } else if constexpr (B == 2) {
    r = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xf, 0x5, false);   // banks 0, 2: row_shl:4 (lane i+4)
    r = __builtin_amdgcn_update_dpp(r, x, 0x114, 0xf, 0xa, false);   // banks 1, 3: row_shr:4 (lane i-4)
  } else {
    r = __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, false);  // row_ror:8 = lane i ^ 8 in a 16-lane row
  }
  return __builtin_bit_cast(float, r);
}

// One butterfly level over lane bit B: of the V values a lane holds, it keeps the half selected by
// its bit B (upper half when set) summed with the partner's same half, sending the other half.
template <int V, int B>
__device__ __forceinline__ void butterfly_level(float* a, int lane) {
  const bool up = (lane >> B) & 1;
#pragma unroll
  for (int j = 0; j < V / 2; ++j) {
    const float keep = up ? a[j + V / 2] : a[j];
    const float send = up ? a[j] : a[j + V / 2];
    a[j] = keep + lane_xor<B>(send);
  }
}

// Sums NV = 2^m per-lane values (m <= 4) over the 64 lanes of a wave with m butterfly levels over lane
// bits 0, 1, 3, 2 and plain exchanges over the remaining bits: about 4 NV instructions instead of
// 16 NV for NV separate reductions.  Returns the lane's total; it is the total of value
// reduce_index<NV>(lane) in every lane whose remaining bits (2 when m < 4, and 4, 5) are zero.
template <int NV>
__device__ __forceinline__ float wave_reduce_multi(float (&a)[NV], int lane) {
  static_assert(NV == 1 || NV == 2 || NV == 4 || NV == 8 || NV == 16, "NV must be 2^m, m <= 4");
  if constexpr (NV >= 2) butterfly_level<NV, 0>(a, lane);
  if constexpr (NV >= 4) butterfly_level<NV / 2, 1>(a, lane);
  if constexpr (NV >= 8) butterfly_level<NV / 4, 3>(a, lane);
  if constexpr (NV >= 16) butterfly_level<NV / 8, 2>(a, lane);
  float v = a[0];
  if constexpr (NV < 16) v += lane_xor<2>(v);
  if constexpr (NV < 8) v += lane_xor<3>(v);
  if constexpr (NV < 4) v += lane_xor<1>(v);
  if constexpr (NV < 2) v += lane_xor<0>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Index of the value whose total wave_reduce_multi<NV> leaves in `lane`, and whether the lane holds
// a total to store (one lane per value).
template <int NV>
__device__ __forceinline__ int reduce_index(int lane) {
  int idx = 0;
  if constexpr (NV >= 2) idx += ((lane >> 0) & 1) * (NV / 2);
  if constexpr (NV >= 4) idx += ((lane >> 1) & 1) * (NV / 4);
  if constexpr (NV >= 8) idx += ((lane >> 3) & 1) * (NV / 8);
  if constexpr (NV >= 16) idx += ((lane >> 2) & 1) * (NV / 16);
  return idx;
}

template <int NV>
__device__ __forceinline__ bool reduce_owner(int lane) {
  int used = 0;
  if constexpr (NV >= 2) used |= 1;
  if constexpr (NV >= 4) used |= 2;
  if constexpr (NV >= 8) used |= 8;
  if constexpr (NV >= 16) used |= 4;
  return (lane & ~used) == 0;
}

__host__ __device__ constexpr int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p *= 2;
  return p;
}

// Long filters (K > 12): direct form (symmetric taps give the same values unfolded).
template <typename R, int NPOL, int RB, int THREADS>
__device__ __forceinline__ void fir_adj_generic(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out, int lo,
                                                int hi, int K, const cx_t<R>* __restrict__ h) {
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
        for (int p = 0; p < NPOL; ++p) cmac_conj(acc[r][p], hk, in[(base + r + k) * NPOL + p]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (base + r < hi) store_sample<R, NPOL>(out + (base + r) * NPOL, acc[r]);
  }
}

// acc_k += g conj(y): the conjugate-linear product used by the tap gradient.
template <typename V>
__device__ __forceinline__ void cmac_yconj(V& acc, V g, V y) {
  acc.x = fma(g.x, y.x, acc.x);
  acc.x = fma(g.y, y.y, acc.x);
  acc.y = fma(g.y, y.x, acc.y);
  acc.y = fma(-g.x, y.y, acc.y);
}

// Stores the wave totals of a thread's tap accumulators as FP64 partials red[wave * ldr + col0 + K + k]:
// SYM, the K + 1 folded sums g_k (see the top of the file), columns K + k and K - k both receiving
// g_k / 2 (g_0 whole); otherwise the 2K + 1 sums of k = -K..K.
template <typename R, int K, bool SYM>
__device__ __forceinline__ void tap_wave_sums(const cx_t<R>* acc, double2* __restrict__ red, int ldr, int col0) {
  constexpr int NA = SYM ? K + 1 : 2 * K + 1;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  double* redd = reinterpret_cast<double*>(red);
  constexpr int NV = pow2_at_least(2 * NA);
  if constexpr (sizeof(R) == 4 && NV <= 16) {
    // all 2 NA components reduced together; value 2a + c is component c of accumulator a
    float vals[NV];
#pragma unroll
    for (int a = 0; a < NV / 2; ++a) {
      vals[2 * a] = a < NA ? acc[a].x : 0.f;
      vals[2 * a + 1] = a < NA ? acc[a].y : 0.f;
    }
    const float tot = wave_reduce_multi<NV>(vals, lane);
    const int idx = reduce_index<NV>(lane);
    if (reduce_owner<NV>(lane) && idx < 2 * NA) {
      const int a = idx >> 1, comp = idx & 1;
      if constexpr (SYM) {
        const double v = (a == 0 ? 1.0 : 0.5) * static_cast<double>(tot);
        redd[2 * (wv * ldr + col0 + K + a) + comp] = v;
        redd[2 * (wv * ldr + col0 + K - a) + comp] = v;
      } else {
        redd[2 * (wv * ldr + col0 + a) + comp] = static_cast<double>(tot);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const R sx = wave_sum_last(acc[k].x);
      const R sy = wave_sum_last(acc[k].y);
      if (lane == kLastLane) {
        if constexpr (SYM) {
          const double f = k == 0 ? 1.0 : 0.5;
          const double2 v{f * static_cast<double>(sx), f * static_cast<double>(sy)};
          red[wv * ldr + col0 + K + k] = v;
          red[wv * ldr + col0 + K - k] = v;
        } else {
          red[wv * ldr + col0 + k] = double2{static_cast<double>(sx), static_cast<double>(sy)};
        }
      }
    }
  }
}

// FIR adjoint and tap correlation of one step in a single pass, RB outputs per thread from one register
// window of G_u (reads in[lo-K, hi+RB+K-2]):
//   G_x,p = sum_k conj(h_k) G_u,(p+k)                               for p in [lo, hi), into out
//   a_k  += G_u,(p+k) conj(y_p), k = -K..K                          for p in [own_lo, own_hi)
// with y_p = yprev[p + yshift].  Over all tiles, sum_{owned p} G_u,(p+k) conj(y_p) is the tap
// correlation sum_m G_u,m conj(y_(m-k)) (every position of the circle is owned by one tile; only the
// grouping of the terms differs).  SYM: both products take the pair sums G_u,(p+k) + G_u,(p-k) once,
// a_k being the folded sum g_k.  Halo positions weight finite G_u by y = 0; positions past hi, whose
// windows reach LDS past the computed range, are skipped.
template <typename R, int NPOL, int RB, int THREADS, int K, bool SYM>
__device__ __forceinline__ void fir_adj_tap_fixed(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out, int lo,
                                                  int hi, const cx_t<R>* __restrict__ h, int own_lo, int own_hi,
                                                  const cx_t<R>* __restrict__ yprev, int yshift,
                                                  double2* __restrict__ red, int ldr, int col0) {
  using V = cx_t<R>;
  constexpr int W = RB + 2 * K;
  constexpr int NA = SYM ? K + 1 : 2 * K + 1;
  V ta[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) ta[k] = V{0, 0};
  for (int base = lo + static_cast<int>(threadIdx.x) * RB; base < hi; base += THREADS * RB) {
    V win[W][NPOL];
#pragma unroll
    for (int j = 0; j < W; ++j) load_sample<R, NPOL>(in + (base - K + j) * NPOL, win[j]);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int p = base + r;
      if (p >= hi) continue;
      V y[NPOL];
      if (p >= own_lo && p < own_hi) {
        load_sample<R, NPOL>(yprev + (p + yshift) * NPOL, y);
      } else {
#pragma unroll
        for (int q = 0; q < NPOL; ++q) y[q] = V{0, 0};
      }
      V o[NPOL];
#pragma unroll
      for (int q = 0; q < NPOL; ++q) {
        o[q] = V{0, 0};
        if constexpr (SYM) {
          const V g0 = win[r + K][q];
          cmac_conj(o[q], h[K], g0);
          cmac_yconj(ta[0], g0, y[q]);
#pragma unroll
          for (int k = 1; k <= K; ++k) {
            const V a = win[r + K + k][q], b = win[r + K - k][q];
            const V ps{a.x + b.x, a.y + b.y};
            cmac_conj(o[q], h[K + k], ps);
            cmac_yconj(ta[k], ps, y[q]);
          }
        } else {
#pragma unroll
          for (int k = -K; k <= K; ++k) {
            const V g = win[r + K + k][q];
            cmac_conj(o[q], h[K + k], g);
            cmac_yconj(ta[K + k], g, y[q]);
          }
        }
      }
      store_sample<R, NPOL>(out + p * NPOL, o);
    }
  }
  tap_wave_sums<R, K, SYM>(ta, red, ldr, col0);
}

// Long filters (K > 12): one tap at a time over the owned positions j, sum_j G_u,j conj(y_(j-k)); with
// sym the mirrored pair is summed and halved as in tap_wave_sums.
template <typename R, int NPOL, int RB2, int THREADS>
__device__ __forceinline__ void tapgrad_generic(const cx_t<R>* __restrict__ gu, int own_lo, int Lw, int K,
                                                const cx_t<R>* __restrict__ yprev, int yshift,
                                                double2* __restrict__ red, int ldr, int col0, bool sym) {
  using V = cx_t<R>;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int own_hi = own_lo + Lw;
  for (int k = sym ? 0 : -K; k <= K; ++k) {
    V acc{0, 0};
    for (int j = own_lo + static_cast<int>(threadIdx.x); j < own_hi; j += THREADS)
#pragma unroll
      for (int p = 0; p < NPOL; ++p) {
        V y = yprev[(j + yshift - k) * NPOL + p];
        if (sym && k > 0) {
          const V b = yprev[(j + yshift + k) * NPOL + p];
          y = V{y.x + b.x, y.y + b.y};
        }
        cmac_yconj(acc, gu[j * NPOL + p], y);
      }
    const R sx = wave_sum_last(acc.x);
    const R sy = wave_sum_last(acc.y);
    if (lane == kLastLane) {
      const double f = (sym && k > 0) ? 0.5 : 1.0;
      const double2 v{f * static_cast<double>(sx), f * static_cast<double>(sy)};
      red[wv * ldr + col0 + K + k] = v;
      if (sym) red[wv * ldr + col0 + K - k] = v;
    }
  }
}

template <typename R, int NPOL, int RB, int RB2, int THREADS, bool SYM, int KMAX>
__device__ __forceinline__ void adj_step_dispatch_t(const cx_t<R>* gb, cx_t<R>* ga, int lo, int hi, int K,
                                                    const cx_t<R>* h, int own_lo, int Lw, const cx_t<R>* yprev,
                                                    int yshift, double2* red, int ldr, int col0) {
  switch (K) {
#define LDBP_BWD_CASE(k)                                                                             \
  case k:                                                                                            \
    if constexpr (k <= KMAX) {                                                                       \
      fir_adj_tap_fixed<R, NPOL, RB, THREADS, k, SYM>(gb, ga, lo, hi, h, own_lo, own_lo + Lw, yprev, yshift, \
                                                     red, ldr, col0);                                \
    } else {                                                                                         \
      fir_adj_generic<R, NPOL, RB, THREADS>(gb, ga, lo, hi, K, h);                                   \
      tapgrad_generic<R, NPOL, RB2, THREADS>(gb, own_lo, Lw, K, yprev, yshift, red, ldr, col0, SYM); \
    }                                                                                                \
    break;
    LDBP_BWD_CASE(0) LDBP_BWD_CASE(1) LDBP_BWD_CASE(2) LDBP_BWD_CASE(3)
    LDBP_BWD_CASE(4) LDBP_BWD_CASE(5) LDBP_BWD_CASE(6) LDBP_BWD_CASE(7)
    LDBP_BWD_CASE(8) LDBP_BWD_CASE(9) LDBP_BWD_CASE(10) LDBP_BWD_CASE(11)
    LDBP_BWD_CASE(12)
#undef LDBP_BWD_CASE
    default:
      fir_adj_generic<R, NPOL, RB, THREADS>(gb, ga, lo, hi, K, h);
      tapgrad_generic<R, NPOL, RB2, THREADS>(gb, own_lo, Lw, K, yprev, yshift, red, ldr, col0, SYM);
      break;
  }
}

template <typename R, int NPOL, int RB, int RB2, int THREADS, int KMAX>
__device__ __forceinline__ void adj_step_dispatch(const cx_t<R>* gb, cx_t<R>* ga, int lo, int hi, int K,
                                                  const cx_t<R>* h, int own_lo, int Lw, const cx_t<R>* yprev,
                                                  int yshift, double2* red, int ldr, int col0, bool sym) {
  if (sym)
    adj_step_dispatch_t<R, NPOL, RB, RB2, THREADS, true, KMAX>(gb, ga, lo, hi, K, h, own_lo, Lw, yprev, yshift, red,
                                                               ldr, col0);
  else
    adj_step_dispatch_t<R, NPOL, RB, RB2, THREADS, false, KMAX>(gb, ga, lo, hi, K, h, own_lo, Lw, yprev, yshift, red,
                                                                ldr, col0);
}

// Up to kMaxBwdTiles tiles of the block's inputs loaded with all their global loads in flight before the
// first LDS store, so the tile waits for one round trip instead of one per buffer: tile i is
// src[i] over the circular positions [t0 - halo[i], t0 - halo[i] + width[i]) into dst[i].
constexpr int kMaxBwdTiles = 5;   // block input, output gradient and up to 3 stored step outputs
template <typename R>
struct BwdTile {
  const cx_t<R>* src;
  cx_t<R>* dst;
  int halo, width;
};

template <typename R, int NPOL, int THREADS, int NT>
__device__ __forceinline__ void load_bwd_tiles(const BwdTile<R> (&t)[kMaxBwdTiles], int cnt, int n, int t0,
                                               bool general) {
  using V = cx_t<R>;
  // 64 bytes of samples per tile and thread in flight; with more than two tiles, 32 bytes for samples of
  // 16 bytes or more (the registers stay under 48)
  constexpr int kLoadBatch = 64 / static_cast<int>(sizeof(V) * NPOL) / (NT > 2 && sizeof(V) * NPOL >= 16 ? 2 : 1);
  // one addition or subtraction brings t0 - halo + j onto the circle unless the halo exceeds n (tiny
  // waveforms), which takes the remainder
  auto wrap = [n, general](int g) {
    if (general) {
      g %= n;
      return g < 0 ? g + n : g;
    }
    return g < 0 ? g + n : (g >= n ? g - n : g);
  };
  int W = 0;
#pragma unroll
  for (int i = 0; i < NT; ++i)
    if (i < cnt) W = max(W, t[i].width);
  for (int j0 = threadIdx.x; j0 < W; j0 += kLoadBatch * THREADS) {
    V v[NT][kLoadBatch][NPOL];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (i < cnt) {
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
          const int j = min(j0 + u * THREADS, t[i].width - 1);  // past the end: reload the last sample, not stored
          load_sample<R, NPOL>(t[i].src + static_cast<int64_t>(wrap(t0 - t[i].halo + j)) * NPOL, v[i][u]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (i < cnt) {
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
          const int j = j0 + u * THREADS;
          if (j < t[i].width) store_sample<R, NPOL>(t[i].dst + j * NPOL, v[i][u]);
        }
      }
    }
  }
}

// Buffer margin of Y_s (block output of step s within the tile's recompute): the forward starts from
// a margin of 2H and each step shrinks the valid margin by K_s + kappa_s; a filtered step keeps its
// FIR output (margin V_{s-1} - K_s) in place and rotates only the inner part, so the buffer margin of
// Y_s is 2H - h_s + kappa_s with h_s = sum_{i<=s} (K_i + kappa_i).  Mirrored by bwd_lds_bytes().
__host__ __device__ inline int bwd_y_width(int Lw, int H, int hs, int kap = 0) { return Lw + 4 * H - 2 * hs + 2 * kap; }

// Whether the backward keeps G_B in the buffer of the block output Y_S (see the kernel's carve-up).
__host__ __device__ constexpr bool bwd_gb_in_ys(bool filtered, int npol) { return !filtered && npol == 2; }

// Sum over the tile's own positions of q_i P_{i-k} for every k in [-kap, kap] (the power-filter tap
// correlation of a filtered step), one wave reduction per tap into red columns col0 + kap + k.
template <typename R>
__device__ __forceinline__ void eta_grad(const R* __restrict__ Q, const R* __restrict__ PP, int own_lo, int Lw,
                                         int kap, double2* __restrict__ red, int ldr, int col0, int threads) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int k = -kap; k <= kap; ++k) {
    R acc = 0;
    for (int i = own_lo + static_cast<int>(threadIdx.x); i < own_lo + Lw; i += threads) acc = fma(Q[i], PP[i - k], acc);
    acc = wave_sum_last(acc);
    if (lane == kLastLane) red[wv * ldr + col0 + kap + k] = double2{static_cast<double>(acc), 0.0};
  }
}

// Zeroed entries of Q and PP past the filled range, read by the fixed-kappa windows (RBF - 1 of them at
// most); they fit in the arrays' padding for complex64 (pad 8).
constexpr int kFiltTail = 8;

// Adjoint of the filtered phase of one step over G indices [lo + kap, hi - kap), with q = dL/dphi in Q
// and P = |y|^2 in PP, both filled on [lo, hi):
//   F_i = sum_k eta_k P_{i-k},  r_i = c sum_k eta_k q_{i+k},  G_u,i = (G_y,i + 2 r_i y_i) e^{-j c F_i};
// y_i is ycur[(i + yoff) * NPOL + p].  Returns this thread's share of sum_{owned i} q_i F_i (dL/dc).
// Generic kappa: one sample per thread and iteration.
template <typename R, int NPOL, int THREADS>
__device__ __forceinline__ R nl_adjoint_generic(const cx_t<R>* __restrict__ ycur, int yoff, const cx_t<R>* __restrict__ GA,
                                                cx_t<R>* __restrict__ GB, const R* __restrict__ Q,
                                                const R* __restrict__ PP, int lo, int hi, int kap,
                                                const R* __restrict__ e, R cr, R coef, int own_lo, int own_hi) {
  using V = cx_t<R>;
  R accc = 0;
  for (int i = lo + kap + static_cast<int>(threadIdx.x); i < hi - kap; i += THREADS) {
    R F = 0, r = 0;
    for (int k = -kap; k <= kap; ++k) {
      F = fma(e[kap + k], PP[i - k], F);
      r = fma(e[kap + k], Q[i + k], r);
    }
    R sn, co;
    phase_sincos(coef, F, sn, co);
    const R tr = 2 * cr * r;
#pragma unroll
    for (int pp = 0; pp < NPOL; ++pp) {
      const V yv = ycur[(i + yoff) * NPOL + pp];
      const V gv = GA[i * NPOL + pp];
      // G_y e^{-j phi} + 2 r u with u = y e^{-j phi}: (G_y + 2 r y) e^{-j phi}
      const R tx = gv.x + tr * yv.x;
      const R ty = gv.y + tr * yv.y;
      GB[i * NPOL + pp] = V{tx * co + ty * sn, ty * co - tx * sn};
    }
    if (i >= own_lo && i < own_hi) accc += Q[i] * F;
  }
  return accc;
}

// Fixed kappa: RBF (odd) consecutive samples per thread from register windows of P and q (2 (RBF + 2 kappa)
// LDS reads for RBF samples instead of 2 (2 kappa + 1) each), the filter taps uniform (scalar
// registers).  Windows reach up to hi + RBF - 2; the caller zeroes Q and PP on [hi, hi + kFiltTail), so
// no LDS left over from other data enters a sum.
template <typename R, int NPOL, int THREADS, int KAP>
__device__ __forceinline__ R nl_adjoint_fixed(const cx_t<R>* __restrict__ ycur, int yoff, const cx_t<R>* __restrict__ GA,
                                              cx_t<R>* __restrict__ GB, const R* __restrict__ Q,
                                              const R* __restrict__ PP, int lo, int hi, const R* __restrict__ e,
                                              R cr, R coef, int own_lo, int own_hi) {
  using V = cx_t<R>;
  constexpr int RBF = 7;  // odd: lanes RBF words apart fall on distinct LDS banks
  static_assert(RBF - 1 <= kFiltTail, "windows must stay inside the zeroed tail");
  constexpr int W = RBF + 2 * KAP;
  R accc = 0;
  const int lo2 = lo + KAP, hi2 = hi - KAP;
  for (int base = lo2 + static_cast<int>(threadIdx.x) * RBF; base < hi2; base += THREADS * RBF) {
    // F from a window of P, then r from a window of q (one window live at a time)
    R F[RBF], rr[RBF], qo[RBF];
    {
      R w[W];
#pragma unroll
      for (int j = 0; j < W; ++j) w[j] = PP[base - KAP + j];
#pragma unroll
      for (int r = 0; r < RBF; ++r) F[r] = 0;
#pragma unroll
      for (int k = -KAP; k <= KAP; ++k) {
        const R ek = e[KAP + k];
#pragma unroll
        for (int r = 0; r < RBF; ++r) F[r] = fma(ek, w[r - k + KAP], F[r]);
      }
    }
    {
      R w[W];
#pragma unroll
      for (int j = 0; j < W; ++j) w[j] = Q[base - KAP + j];
#pragma unroll
      for (int r = 0; r < RBF; ++r) {
        rr[r] = 0;
        qo[r] = w[r + KAP];
      }
#pragma unroll
      for (int k = -KAP; k <= KAP; ++k) {
        const R ek = e[KAP + k];
#pragma unroll
        for (int r = 0; r < RBF; ++r) rr[r] = fma(ek, w[r + k + KAP], rr[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RBF; ++r) {
      const int i = base + r;
      if (i < hi2) {
        R sn, co;
        phase_sincos(coef, F[r], sn, co);
        const R tr = 2 * cr * rr[r];
#pragma unroll
        for (int pp = 0; pp < NPOL; ++pp) {
          const V yv = ycur[(i + yoff) * NPOL + pp];
          const V gv = GA[i * NPOL + pp];
          const R tx = gv.x + tr * yv.x;
          const R ty = gv.y + tr * yv.y;
          GB[i * NPOL + pp] = V{tx * co + ty * sn, ty * co - tx * sn};
        }
        if (i >= own_lo && i < own_hi) accc += qo[r] * F[r];
      }
    }
  }
  return accc;
}

template <typename R, int NPOL, int THREADS>
__device__ __forceinline__ R nl_adjoint_dispatch(const cx_t<R>* ycur, int yoff, const cx_t<R>* GA, cx_t<R>* GB,
                                                 const R* Q, const R* PP, int lo, int hi, int kap, const R* e, R cr,
                                                 R coef, int own_lo, int own_hi) {
  if constexpr (sizeof(R) == 4) {
    switch (kap) {
#define LDBP_NLA_CASE(k) \
  case k: return nl_adjoint_fixed<R, NPOL, THREADS, k>(ycur, yoff, GA, GB, Q, PP, lo, hi, e, cr, coef, own_lo, own_hi);
      LDBP_NLA_CASE(0) LDBP_NLA_CASE(1) LDBP_NLA_CASE(2) LDBP_NLA_CASE(3) LDBP_NLA_CASE(4) LDBP_NLA_CASE(5) LDBP_NLA_CASE(6)
      LDBP_NLA_CASE(8) LDBP_NLA_CASE(10) LDBP_NLA_CASE(12) LDBP_NLA_CASE(16) LDBP_NLA_CASE(20)
#undef LDBP_NLA_CASE
      default: break;
    }
  }
  return nl_adjoint_generic<R, NPOL, THREADS>(ycur, yoff, GA, GB, Q, PP, lo, hi, kap, e, cr, coef, own_lo, own_hi);
}

// Filter-tap gradient sums g_k = sum_{owned i} q_i P_{i-k}, k = -kap..kap, for fixed kappa: RBF owned
// samples per thread against a register window of P, the 2 kappa + 1 sums reduced over the wave in
// groups of 16 by the butterfly (wave_reduce_multi) and stored as wave partials red[wv][col0 + k + kap].
template <typename R, int THREADS, int KAP>
__device__ __forceinline__ void eta_grad_fixed(const R* __restrict__ Q, const R* __restrict__ PP, int own_lo, int Lw,
                                               double2* __restrict__ red, int ldr, int col0) {
  constexpr int RBF = 7;  // odd: lanes RBF words apart fall on distinct LDS banks
  static_assert(RBF - 1 <= kFiltTail, "windows must stay inside the zeroed tail");
  constexpr int NE = 2 * KAP + 1;
  constexpr int W = RBF + 2 * KAP;
  const int own_hi = own_lo + Lw;
  R g[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) g[k] = 0;
  for (int base = own_lo + static_cast<int>(threadIdx.x) * RBF; base < own_hi; base += THREADS * RBF) {
    R wp[W], q[RBF];
#pragma unroll
    for (int j = 0; j < W; ++j) wp[j] = PP[base - KAP + j];   // below hi + kFiltTail (zeroed beyond hi)
#pragma unroll
    for (int r = 0; r < RBF; ++r) q[r] = base + r < own_hi ? Q[base + r] : R(0);
#pragma unroll
    for (int k = -KAP; k <= KAP; ++k)
#pragma unroll
      for (int r = 0; r < RBF; ++r) g[KAP + k] = fma(q[r], wp[r - k + KAP], g[KAP + k]);
  }
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int g0 = 0; g0 < NE; g0 += 16) {
    float vals[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) vals[j] = g0 + j < NE ? g[g0 + j] : 0.f;
    const float tot = wave_reduce_multi<16>(vals, lane);
    const int idx = g0 + reduce_index<16>(lane);
    if (reduce_owner<16>(lane) && idx < NE) red[wv * ldr + col0 + idx] = double2{static_cast<double>(tot), 0.0};
  }
}

template <typename R, int THREADS>
__device__ __forceinline__ void eta_grad_dispatch(const R* Q, const R* PP, int own_lo, int Lw, int kap,
                                                  double2* red, int ldr, int col0) {
  if constexpr (sizeof(R) == 4) {
    switch (kap) {
#define LDBP_EG_CASE(k) \
  case k: eta_grad_fixed<R, THREADS, k>(Q, PP, own_lo, Lw, red, ldr, col0); return;
      LDBP_EG_CASE(0) LDBP_EG_CASE(1) LDBP_EG_CASE(2) LDBP_EG_CASE(3) LDBP_EG_CASE(4) LDBP_EG_CASE(5) LDBP_EG_CASE(6)
      LDBP_EG_CASE(8) LDBP_EG_CASE(10) LDBP_EG_CASE(12) LDBP_EG_CASE(16) LDBP_EG_CASE(20)
#undef LDBP_EG_CASE
      default: break;
    }
  }
  eta_grad<R>(Q, PP, own_lo, Lw, kap, red, ldr, col0, THREADS);
}

// FILT: the block's nonlinear steps filter the power (generalised ESSM, eta != NULL); a separate
// instantiation keeps the plain LDBP kernel unchanged.  KMAX: the largest filter half-length of the
// block with fixed-window code compiled in (the host picks the smallest variant that covers the block).
template <typename R, int NPOL, int RB, int RB2, int THREADS, bool FILT, int KMAX = 12>
__global__ __launch_bounds__(THREADS) void ldbp_bwd_kernel(
    const cx_t<R>* __restrict__ xb, const cx_t<R>* __restrict__ gout, cx_t<R>* __restrict__ gin, int32_t n,
    int32_t tile_len, int32_t ntiles, const cx_t<R>* __restrict__ taps, const R* __restrict__ c, PassTable pt,
    int32_t pad, double2* __restrict__ part, int32_t ncols, int32_t ccol_base, int32_t sym,
    const R* __restrict__ eta, int32_t ecol_base, const cx_t<R>* __restrict__ ys, int64_t ys_stride,
    int32_t nstored, const cx_t<R>* __restrict__ yout) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = THREADS / 64;

  const int tile = static_cast<int>(blockIdx.x % static_cast<uint32_t>(ntiles));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(ntiles);
  const int t0 = tile * tile_len;
  const int Lw = min(tile_len, n - t0);
  const int H = pt.halo;
  const int S = pt.nstep;
  const int ntap_blk = pt.tapoff[S - 1] + 2 * pt.K[S - 1] + 1 - pt.tapoff[0];
  const int neta_blk = FILT ? pt.etaoff[S - 1] + 2 * pt.kap[S - 1] + 1 - pt.etaoff[0] : 0;
  const int ldr = ntap_blk + neta_blk + S;
  auto kapp = [&](int s) { return FILT ? pt.kap[s - 1] : 0; };  // kappa of step s (1-based)

  // LDS carve-up: red (FP64 partials) | Y_0 .. Y_S | GA [| GB | Q | PP]; Y_s has width
  // bwd_y_width(Lw, H, h_s, kappa_s) + pad.
  double2* red = reinterpret_cast<double2*>(smem);
  V* Y0 = reinterpret_cast<V*>(smem + static_cast<size_t>(NW) * ldr * sizeof(double2));
  size_t ytot = 0, ylast = 0;
  {
    int h = 0;
    for (int s = 0; s <= S; ++s) {
      const int kp = s > 0 ? kapp(s) : 0;
      if (s > 0) h += pt.K[s - 1] + kp;
      ylast = ytot;
      ytot += static_cast<size_t>(bwd_y_width(Lw, H, h, kp) + pad) * NPOL;
    }
  }
  V* GA = Y0 + ytot;
  // Unfiltered steps, two polarisations: GB shares the buffer of Y_S.  The Kerr adjoint of step S
  // reads y_i from Y_S at index i (the reverse sweep starts with h = H, so its offset is zero) and
  // writes G_u,i to GB at the same index, and Y_S is not read again; Y_S is at least Lw + 2H wide,
  // the G range.  The freed LDS makes tiles 25% longer (measured 6% faster on 8 x 2^20 x 2, but 4%
  // slower for one polarisation, which keeps GB apart); filtered steps read y at an offset of kappa,
  // so they keep a buffer of their own.
  constexpr bool kGbInYs = bwd_gb_in_ys(FILT, NPOL);
  V* GB = kGbInYs ? Y0 + ylast : GA + static_cast<size_t>(Lw + 2 * H + pad) * NPOL;
  // filtered steps only: Q over the G range, PP over the recompute range (a Y buffer plus a window)
  R* Q = reinterpret_cast<R*>(GA + 2 * static_cast<size_t>(Lw + 2 * H + pad) * NPOL);
  R* PP = Q + (Lw + 2 * H + pad);
  int hs;

  const V* xw = xb + wave * static_cast<int64_t>(n) * NPOL;
  const V* gw = gout + wave * static_cast<int64_t>(n) * NPOL;
  // the block output read from the next checkpoint: complex64; filtered steps of one polarisation only
  // (the two-polarisation filtered kernel has no registers to spare for a third tile, and the host
  // passes no block output with two polarisations)
  constexpr bool kYout = sizeof(R) == 4 && (!FILT || NPOL == 1);

  // 1. block input, block-output gradient (used in step 3) and, when the forward stored them, the
  // outputs of the block's first nstored steps (unfiltered complex64 steps only), each over the range
  // its recompute would cover, or (yout) the block's output Y_S, which the forward stored as the next
  // block's checkpoint; then the forward recompute of the remaining steps.  A stored output is the
  // value the recompute would give, bit for bit: every forward output is the same sequence of fused
  // operations whatever the tiling.
  {
    BwdTile<R> t[kMaxBwdTiles];
    t[0] = BwdTile<R>{xw, Y0, 2 * H, Lw + 4 * H};
    t[1] = BwdTile<R>{gw, GA, H, Lw + 2 * H};
    int cnt = 2;
    if constexpr (!FILT && sizeof(R) == 4) {
      V* yb = Y0;
      int h = 0;
#pragma unroll
      for (int s = 1; s <= kMaxBwdTiles - 2; ++s) {   // constant indices into t (no private memory)
        if (s <= nstored) {
          yb += static_cast<size_t>(bwd_y_width(Lw, H, h) + pad) * NPOL;
          h += pt.K[s - 1];
          t[1 + s] = BwdTile<R>{ys + (s - 1) * ys_stride + wave * static_cast<int64_t>(n) * NPOL, yb, 2 * H - h,
                                bwd_y_width(Lw, H, h)};
          cnt = 2 + s;
        }
      }
    }
    if constexpr (kYout) {
      // Y_S over global [t0 - H, t0 + Lw + H): its buffer starts kappa_S earlier (filtered steps)
      if (yout && nstored == 0) {
        t[2] = BwdTile<R>{yout + wave * static_cast<int64_t>(n) * NPOL, Y0 + ylast + static_cast<size_t>(kapp(S)) * NPOL,
                          H, bwd_y_width(Lw, H, H)};
        cnt = 3;
      }
    }
    if constexpr (!FILT && sizeof(R) == 4) {
      if (cnt > 2) load_bwd_tiles<R, NPOL, THREADS, kMaxBwdTiles>(t, cnt, n, t0, 2 * H >= n);
      else load_bwd_tiles<R, NPOL, THREADS, 2>(t, cnt, n, t0, 2 * H >= n);
    } else if constexpr (kYout) {
      if (cnt > 2) load_bwd_tiles<R, NPOL, THREADS, 3>(t, cnt, n, t0, 2 * H >= n);
      else load_bwd_tiles<R, NPOL, THREADS, 2>(t, cnt, n, t0, 2 * H >= n);
    } else {
      load_bwd_tiles<R, NPOL, THREADS, 2>(t, cnt, n, t0, 2 * H >= n);
    }
  }
  __syncthreads();
  hs = 0;
  V* ycur = Y0;
  int kprev = 0;  // kappa of the step that produced ycur (its buffer extends kprev beyond the valid part)
  for (int s = 1; s <= S; ++s) {
    const int K = pt.K[s - 1];
    const int kp = kapp(s);
    V* ynext = ycur + static_cast<size_t>(bwd_y_width(Lw, H, hs, kprev) + pad) * NPOL;
    const R coef = c[pt.c0 + s - 1] * phase_coef_scale<R>();
    if (sizeof(R) == 4 && ((!FILT && s <= nstored) || (kYout && yout && s == S))) {
      // loaded above
      hs += K + kp;
      kprev = kp;
      ycur = ynext;
      continue;
    }
    if constexpr (FILT) {
      // FIR output over the buffer of Y_s (valid margin of Y_{s-1} minus K), power into PP, then the
      // filtered phase on the inner part
      const int wout = bwd_y_width(Lw, H, hs + K, 0);
      fir_lin_dispatch<R, NPOL, RB, THREADS>(ycur + (kprev + K) * NPOL, ynext, PP, 0, wout, K,
                                             taps + pt.tapoff[s - 1], sym != 0);
      __syncthreads();
      nl_filter_dispatch<R, NPOL, RB, THREADS>(ynext, PP, kp, wout - kp, kp, eta + pt.etaoff[s - 1], coef);
    } else {
      fir_kerr_dispatch<R, NPOL, RB, THREADS, KMAX>(ycur + K * NPOL, ynext, 0, bwd_y_width(Lw, H, hs + K), K,
                                              taps + pt.tapoff[s - 1], coef, sym != 0);
    }
    __syncthreads();
    hs += K + kp;
    kprev = kp;
    ycur = ynext;
  }
  // 2. the block-output gradient is in GA (loaded with the block input)

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  // 3. reverse sweep
  hs = H;
  for (int s = S; s >= 1; --s) {
    const int K = pt.K[s - 1];
    const int kp = kapp(s);
    const int kpp = s > 1 ? kapp(s - 1) : 0;
    const R cr = c[pt.c0 + s - 1];
    const R coef = cr * phase_coef_scale<R>();
    // G_y,s is held over GA indices [H - h_s, H + Lw + h_s); Y_s index = i + yoff with the buffer
    // margin 2H - h_s + kappa_s, so yoff = H - h_s + kappa_s
    const int lo = H - hs, hi = H + Lw + hs, yoff = H - hs + kp;
    const int hprev = hs - K - kp;
    V* yprev = ycur - static_cast<size_t>(bwd_y_width(Lw, H, hprev, kpp) + pad) * NPOL;
    R accc = 0;
    if constexpr (FILT) {
      // q = dL/dphi and P = |y|^2 over the whole G_y range, then the adjoint of the filtered phase over
      // the range shrunk by kappa: G_u = G_y e^{-j phi} + 2 r u, r_i = c sum_k eta_k q_{i+k}
      for (int i = lo + static_cast<int>(threadIdx.x); i < hi; i += THREADS) {
        R pw = 0, q = 0;
        V yv[NPOL], gv[NPOL];
        load_sample<R, NPOL>(ycur + (i + yoff) * NPOL, yv);
        load_sample<R, NPOL>(GA + i * NPOL, gv);
#pragma unroll
        for (int pp = 0; pp < NPOL; ++pp) {
          pw = add_power(pw, yv[pp]);
          q += gv[pp].y * yv[pp].x - gv[pp].x * yv[pp].y;
        }
        Q[i] = q;
        PP[i] = pw;
      }
      if constexpr (sizeof(R) == 4) {
        if (static_cast<int>(threadIdx.x) < kFiltTail) {
          Q[hi + threadIdx.x] = 0;
          PP[hi + threadIdx.x] = 0;
        }
      }
      __syncthreads();
      accc = nl_adjoint_dispatch<R, NPOL, THREADS>(ycur, yoff, GA, GB, Q, PP, lo, hi, kp, eta + pt.etaoff[s - 1], cr,
                                                   coef, H, H + Lw);
      eta_grad_dispatch<R, THREADS>(Q, PP, H, Lw, kp, red, ldr, ntap_blk + pt.etaoff[s - 1] - pt.etaoff[0]);
    } else {
      for (int i = lo + static_cast<int>(threadIdx.x); i < hi; i += THREADS) {
        V yv[NPOL], gv[NPOL];
        R pw = 0, q = 0;
        load_sample<R, NPOL>(ycur + (i + yoff) * NPOL, yv);
        load_sample<R, NPOL>(GA + i * NPOL, gv);
#pragma unroll
        for (int pp = 0; pp < NPOL; ++pp) {
          pw = add_power(pw, yv[pp]);
          q += gv[pp].y * yv[pp].x - gv[pp].x * yv[pp].y;
        }
        R sn, co;
        phase_sincos(coef, pw, sn, co);
        const R tq = 2 * cr * q;
        V gb[NPOL];
#pragma unroll
        for (int pp = 0; pp < NPOL; ++pp) {
          const R tx = gv[pp].x + tq * yv[pp].x;
          const R ty = gv[pp].y + tq * yv[pp].y;
          gb[pp] = V{tx * co + ty * sn, ty * co - tx * sn};
        }
        store_sample<R, NPOL>(GB + i * NPOL, gb);
        if (i >= H && i < H + Lw) accc += q * pw;
      }
    }
    accc = wave_sum_last(accc);
    if (lane == kLastLane) red[wv * ldr + ntap_blk + neta_blk + (s - 1)] = double2{static_cast<double>(accc), 0.0};
    __syncthreads();
    // FIR adjoint into GA over [H - h_{s-1}, H + Lw + h_{s-1}); tap gradient over the owned range.  Y_{s-1}
    // index = GA index + (H - h_{s-1} + kappa_{s-1})
    adj_step_dispatch<R, NPOL, RB, RB2, THREADS, KMAX>(GB, GA, H - hprev, H + Lw + hprev, K, taps + pt.tapoff[s - 1], H,
                                                 Lw, yprev, H - hprev + kpp, red, ldr,
                                                 pt.tapoff[s - 1] - pt.tapoff[0], sym != 0);
    __syncthreads();
    hs = hprev;
    ycur = yprev;
  }

  // 4. block-input gradient and the tile's partial sums
  if (gin) {
    V* gi = gin + wave * static_cast<int64_t>(n) * NPOL;
    for (int j = threadIdx.x; j < Lw; j += THREADS) {
      V v[NPOL];
      load_sample<R, NPOL>(GA + (H + j) * NPOL, v);
      store_sample<R, NPOL>(gi + static_cast<int64_t>(t0 + j) * NPOL, v);
    }
  }
  double2* prow = part + static_cast<int64_t>(blockIdx.x) * ncols;
  for (int col = threadIdx.x; col < ldr; col += THREADS) {
    double sx = 0, sy = 0;
    for (int w = 0; w < NW; ++w) {
      sx += red[w * ldr + col].x;
      sy += red[w * ldr + col].y;
    }
    int g;
    if (col < ntap_blk) {
      g = pt.tapoff[0] + col;
    } else if (col < ntap_blk + neta_blk) {
      // eta_k gradient: the sums above times c of the step
      const int ec = col - ntap_blk;
      int st = 0;
      while (st + 1 < S && pt.etaoff[st + 1] - pt.etaoff[0] <= ec) ++st;
      sx *= static_cast<double>(c[pt.c0 + st]);
      g = ecol_base + pt.etaoff[0] + ec;
    } else {
      g = ccol_base + pt.c0 + (col - ntap_blk - neta_blk);
    }
    prow[g] = double2{sx, sy};
  }
}

// Sums part[tile][col] over tiles in a fixed order; one workgroup per column.
// Deterministic reduction of the per-tile partial sums part[tile][col] in two fixed-order stages.
// Stage 1: block (column group of 16, chunk of kReduceRows tiles); thread (g, c) sums tiles
// chunk*kReduceRows + g + 16 j in increasing j, so each row of 16 columns is one 256-byte read, then
// the 16 row lanes are added in order g = 0..15 into chunk_sums[chunk][col].
constexpr int kReduceRows = 256;

__global__ __launch_bounds__(256) void ldbp_grad_reduce_chunks(const double2* __restrict__ part, int64_t ntiles,
                                                               int32_t ncols, double2* __restrict__ chunk_sums) {
  __shared__ double2 acc[16][17];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + c;
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * kReduceRows;
  const int64_t t1 = min(t0 + kReduceRows, ntiles);
  double ax = 0, ay = 0;
  if (col < ncols) {
    for (int64_t t = t0 + g; t < t1; t += 16) {
      const double2 v = part[t * ncols + col];
      ax += v.x;
      ay += v.y;
    }
  }
  acc[g][c] = double2{ax, ay};
  __syncthreads();
  if (g == 0 && col < ncols) {
    double sx = 0, sy = 0;
    for (int k = 0; k < 16; ++k) {
      sx += acc[k][c].x;
      sy += acc[k][c].y;
    }
    chunk_sums[static_cast<int64_t>(blockIdx.y) * ncols + col] = double2{sx, sy};
  }
}

// Stage 2: one thread per column adds the chunk sums in chunk order and stores the gradient
// (columns: taps, then power filters, then Kerr coefficients).
template <typename R>
__global__ __launch_bounds__(256) void ldbp_grad_reduce(const double2* __restrict__ chunk_sums, int64_t nchunks,
                                                        int32_t ncols, int32_t ntaps, cx_t<R>* __restrict__ gtaps,
                                                        R* __restrict__ gc, int32_t neta, R* __restrict__ geta) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= ncols) return;
  double sx = 0, sy = 0;
  for (int64_t k = 0; k < nchunks; ++k) {
    const double2 v = chunk_sums[k * ncols + col];
    sx += v.x;
    sy += v.y;
  }
  if (col < ntaps) gtaps[col] = cx_t<R>{static_cast<R>(sx), static_cast<R>(sy)};
  else if (col < ntaps + neta) geta[col - ntaps] = static_cast<R>(sx);
  else gc[col - ntaps - neta] = static_cast<R>(sx);
}

// ---------------------------------------------------------------- host side

template <typename R, int NPOL> struct BwdCfg;
// Odd window widths keep the lanes' LDS reads on distinct banks.
template <> struct BwdCfg<float, 1> { static constexpr int RB = 5, RB2 = 5, THREADS = 256; };
template <> struct BwdCfg<float, 2> { static constexpr int RB = 3, RB2 = 3, THREADS = 256; };
template <> struct BwdCfg<double, 1> { static constexpr int RB = 3, RB2 = 3, THREADS = 256; };
template <> struct BwdCfg<double, 2> { static constexpr int RB = 1, RB2 = 1, THREADS = 256; };

static int bwd_pad(int dtype, int npol) {
  (void)npol;
  return dtype == LDBP_C64 ? 8 : 4;
}

// Waves per backward workgroup: the FP64 partial-sum rows at the start of the LDS, one per wave.
static int bwd_waves(int dtype, int npol) {
  if (dtype == LDBP_C64) return (npol == 2 ? BwdCfg<float, 2>::THREADS : BwdCfg<float, 1>::THREADS) / 64;
  return (npol == 2 ? BwdCfg<double, 2>::THREADS : BwdCfg<double, 1>::THREADS) / 64;
}

int bwd_chunk_capacity(int dtype, int npol) {
  if (dtype == LDBP_C64)
    return npol == 2 ? BwdCfg<float, 2>::RB * BwdCfg<float, 2>::THREADS : BwdCfg<float, 1>::RB * BwdCfg<float, 1>::THREADS;
  return npol == 2 ? BwdCfg<double, 2>::RB * BwdCfg<double, 2>::THREADS
                   : BwdCfg<double, 1>::RB * BwdCfg<double, 1>::THREADS;
}

size_t bwd_lds_bytes(int dtype, int npol, int Lw, const PassTable& pt, bool filtered) {
  const int pad = bwd_pad(dtype, npol);
  const int S = pt.nstep;
  const int ntap_blk = pt.tapoff[S - 1] + 2 * pt.K[S - 1] + 1 - pt.tapoff[0];
  const int neta_blk = filtered ? pt.etaoff[S - 1] + 2 * pt.kap[S - 1] + 1 - pt.etaoff[0] : 0;
  size_t elems = 0;
  int hs = 0;
  for (int s = 0; s <= S; ++s) {
    const int kp = (s > 0 && filtered) ? pt.kap[s - 1] : 0;
    if (s > 0) hs += pt.K[s - 1] + kp;
    elems += static_cast<size_t>(bwd_y_width(Lw, pt.halo, hs, kp) + pad);
  }
  elems += (bwd_gb_in_ys(filtered, npol) ? 1 : 2) * static_cast<size_t>(Lw + 2 * pt.halo + pad);   // GA [and GB]
  size_t reals = 0;
  if (filtered) reals = static_cast<size_t>(Lw + 2 * pt.halo + pad) + static_cast<size_t>(Lw + 4 * pt.halo + pad + 8);
  return static_cast<size_t>(bwd_waves(dtype, npol)) * (ntap_blk + neta_blk + S) * sizeof(double2) +
         elems * npol * cx_size(dtype) +
         reals * real_size(dtype);
}

template <typename R, int NPOL>
static int launch_bwd_block_t(const void* xb, const void* gout, void* gin, int64_t nwave, int32_t n,
                              int32_t tile_len, const PassTable& pt, const void* taps, const void* c, void* part,
                              int32_t ncols, int32_t ccol_base, int sym, const void* eta, int32_t ecol_base,
                              const void* ys, int64_t ys_stride, int32_t nstored, const void* yout,
                              hipStream_t stream) {
  using Cfg = BwdCfg<R, NPOL>;
  const int64_t ntiles = (n + tile_len - 1) / tile_len;
  const int64_t nblocks = ntiles * nwave;
  if (nblocks > 0x7fffffffLL) return fail(LDBP_EUNSUPPORTED, "grid too large");
  const size_t lds = bwd_lds_bytes(sizeof(R) == 4 ? LDBP_C64 : LDBP_C128, NPOL, tile_len, pt, eta != nullptr);
  int kmax = 0;
  for (int s = 0; s < pt.nstep; ++s) kmax = std::max(kmax, pt.K[s]);
  auto kern = eta ? ldbp_bwd_kernel<R, NPOL, Cfg::RB, Cfg::RB2, Cfg::THREADS, true>
                  : ldbp_bwd_kernel<R, NPOL, Cfg::RB, Cfg::RB2, Cfg::THREADS, false>;
  // complex64 LDBP blocks of short filters: the variants with fewer fixed-window cases use fewer
  // registers (more waves per SIMD)
  if constexpr (sizeof(R) == 4) {
    if (!eta && kmax <= 2) kern = ldbp_bwd_kernel<R, NPOL, Cfg::RB, Cfg::RB2, Cfg::THREADS, false, 2>;
    else if (!eta && kmax <= 7) kern = ldbp_bwd_kernel<R, NPOL, Cfg::RB, Cfg::RB2, Cfg::THREADS, false, 7>;
  }
  if (lds > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(nblocks)), dim3(Cfg::THREADS), lds, stream,
                     static_cast<const cx_t<R>*>(xb), static_cast<const cx_t<R>*>(gout), static_cast<cx_t<R>*>(gin),
                     n, tile_len, static_cast<int32_t>(ntiles), static_cast<const cx_t<R>*>(taps),
                     static_cast<const R*>(c), pt, bwd_pad(sizeof(R) == 4 ? LDBP_C64 : LDBP_C128, NPOL),
                     static_cast<double2*>(part), ncols, ccol_base, sym, static_cast<const R*>(eta), ecol_base,
                     static_cast<const cx_t<R>*>(ys), ys_stride, nstored, static_cast<const cx_t<R>*>(yout));
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

int launch_bwd_block(int dtype, int npol, const void* xb, const void* gout, void* gin, int64_t nwave, int32_t n,
                     int32_t tile_len, const PassTable& pt, const void* taps, const void* c, void* part,
                     int32_t ncols, int32_t ccol_base, int sym, hipStream_t stream, const void* eta,
                     int32_t ecol_base, const void* ys, int64_t ys_stride, int32_t nstored, const void* yout) {
  if (nstored > 0 && (eta || dtype != LDBP_C64 || nstored > kMaxBwdTiles - 2 || nstored > pt.nstep))
    return fail(LDBP_EINVAL, "stored step outputs: %d for a block of %d steps", nstored, pt.nstep);
  if (yout && (dtype != LDBP_C64 || nstored > 0 || (eta && npol != 1)))
    return fail(LDBP_EINVAL, "a stored block output needs complex64 steps, one polarisation when filtered, and no "
                "other stored outputs");
#define LDBP_BWD_ARGS \
  xb, gout, gin, nwave, n, tile_len, pt, taps, c, part, ncols, ccol_base, sym, eta, ecol_base, ys, ys_stride, nstored, \
      yout, stream
  if (dtype == LDBP_C64)
    return npol == 1 ? launch_bwd_block_t<float, 1>(LDBP_BWD_ARGS) : launch_bwd_block_t<float, 2>(LDBP_BWD_ARGS);
  return npol == 1 ? launch_bwd_block_t<double, 1>(LDBP_BWD_ARGS) : launch_bwd_block_t<double, 2>(LDBP_BWD_ARGS);
#undef LDBP_BWD_ARGS
}

int64_t grad_reduce_chunks(int64_t ntiles) { return (ntiles + kReduceRows - 1) / kReduceRows; }

int launch_grad_reduce(int dtype, const void* part, int64_t ntiles, int32_t ncols, int32_t ntaps, void* gtaps,
                       void* gc, hipStream_t stream, int32_t neta, void* geta, void* chunk_sums) {
  const int64_t nchunks = grad_reduce_chunks(ntiles);
  if (nchunks > 65535) return fail(LDBP_EUNSUPPORTED, "too many tiles (%lld) for the gradient reduction", (long long)ntiles);
  hipLaunchKernelGGL(ldbp_grad_reduce_chunks, dim3((ncols + 15) / 16, static_cast<uint32_t>(nchunks)), dim3(256), 0,
                     stream, static_cast<const double2*>(part), ntiles, ncols, static_cast<double2*>(chunk_sums));
  LDBP_HIP_CHECK(hipGetLastError());
  const dim3 grid((ncols + 255) / 256);
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(ldbp_grad_reduce<float>, grid, dim3(256), 0, stream,
                       static_cast<const double2*>(chunk_sums), nchunks, ncols, ntaps, static_cast<float2*>(gtaps),
                       static_cast<float*>(gc), neta, static_cast<float*>(geta));
  else
    hipLaunchKernelGGL(ldbp_grad_reduce<double>, grid, dim3(256), 0, stream,
                       static_cast<const double2*>(chunk_sums), nchunks, ncols, ntaps, static_cast<double2*>(gtaps),
                       static_cast<double*>(gc), neta, static_cast<double*>(geta));
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

}  // namespace ldbp
