// In-LDS Stockham FFT building blocks for gfx950: lengths whose prime factors are 2, 3 and 5.
//
// Data in LDS is laid out as [len][width]: element i of transform w sits at
// i*width + w, so `width` (a power of two) independent transforms of length `len` are done
// together.  A stage of radix RAD with Ns = product of the earlier radices
// reads v_r = in[j + r len/RAD], multiplies by the twiddles W_{Ns RAD}^{r (j mod Ns)},
// takes an RAD-point DFT in registers and writes out[(j/Ns) Ns RAD + (j mod Ns) + r Ns]
// (the self-sorting Stockham formulation; no bit reversal).  Stages ping-pong
// between two buffers; radices are taken as 16, 8, 4 or 2 while the remaining length is even,
// then 3 and 5.  Twiddles come from a table W_len^k, k < len, computed in FP64 and rounded once.
#pragma once

#include "common.h"

namespace ldbp {

// cos/sin(2 pi k / 16), k = 0..4 (exact values of the regular 16-gon)
__device__ constexpr double kC16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                       0.38268343236508977173, 0.0};

template <typename R, int DIR>
__device__ __forceinline__ cx_t<R> w16(int k) {
  // W_16^k = exp(DIR * -2 pi i k / 16), DIR = +1 forward, -1 inverse; k in [0, 16)
  using V = cx_t<R>;
  k &= 15;
  const int q = k >> 2, m = k & 3;
  R c = static_cast<R>(kC16[m]), s = static_cast<R>(kC16[4 - m]);
  // rotate by quarter turns: (c, s) is cos/sin of 2 pi m / 16
  R cr, sr;
  switch (q) {
    case 0: cr = c; sr = s; break;
    case 1: cr = -s; sr = c; break;
    case 2: cr = -c; sr = -s; break;
    default: cr = s; sr = -c; break;
  }
  return V{cr, DIR > 0 ? -sr : sr};
}

// cos and sin of 2 pi / 5 and 4 pi / 5, and sin(2 pi / 3)
__device__ constexpr double kC5_1 = 0.30901699437494742410, kC5_2 = -0.80901699437494742410;
__device__ constexpr double kS5_1 = 0.95105651629515357212, kS5_2 = 0.58778525229247312917;
__device__ constexpr double kS3 = 0.86602540378443864676;

// cos and sin of 2 pi m / R, m < R, for the composite radices 6, 9, 10, 12 and 15
__device__ constexpr double kCos6[6] = {1.0, 5.0e-1, -5.0e-1, -1.0, -5.0e-1, 5.0e-1};
__device__ constexpr double kSin6[6] = {0.0, 8.66025403784438646764e-1, 8.66025403784438646764e-1, 0.0, -8.66025403784438646764e-1, -8.66025403784438646764e-1};
__device__ constexpr double kCos9[9] = {1.0, 7.66044443118978035202e-1, 1.73648177666930348852e-1, -5.0e-1, -9.39692620785908384054e-1, -9.39692620785908384054e-1, -5.0e-1, 1.73648177666930348852e-1, 7.66044443118978035202e-1};
__device__ constexpr double kSin9[9] = {0.0, 6.42787609686539326323e-1, 9.84807753012208059367e-1, 8.66025403784438646764e-1, 3.42020143325668733044e-1, -3.42020143325668733044e-1, -8.66025403784438646764e-1, -9.84807753012208059367e-1, -6.42787609686539326323e-1};
__device__ constexpr double kCos10[10] = {1.0, 8.09016994374947424102e-1, 3.09016994374947424102e-1, -3.09016994374947424102e-1, -8.09016994374947424102e-1, -1.0, -8.09016994374947424102e-1, -3.09016994374947424102e-1, 3.09016994374947424102e-1, 8.09016994374947424102e-1};
__device__ constexpr double kSin10[10] = {0.0, 5.87785252292473129169e-1, 9.51056516295153572116e-1, 9.51056516295153572116e-1, 5.87785252292473129169e-1, 0.0, -5.87785252292473129169e-1, -9.51056516295153572116e-1, -9.51056516295153572116e-1, -5.87785252292473129169e-1};
__device__ constexpr double kCos12[12] = {1.0, 8.66025403784438646764e-1, 5.0e-1, 0.0, -5.0e-1, -8.66025403784438646764e-1, -1.0, -8.66025403784438646764e-1, -5.0e-1, 0.0, 5.0e-1, 8.66025403784438646764e-1};
__device__ constexpr double kSin12[12] = {0.0, 5.0e-1, 8.66025403784438646764e-1, 1.0, 8.66025403784438646764e-1, 5.0e-1, 0.0, -5.0e-1, -8.66025403784438646764e-1, -1.0, -8.66025403784438646764e-1, -5.0e-1};
__device__ constexpr double kCos15[15] = {1.0, 9.13545457642600895502e-1, 6.69130606358858213826e-1, 3.09016994374947424102e-1, -1.045284632676534714e-1, -5.0e-1, -8.09016994374947424102e-1, -9.78147600733805637929e-1, -9.78147600733805637929e-1, -8.09016994374947424102e-1, -5.0e-1, -1.045284632676534714e-1, 3.09016994374947424102e-1, 6.69130606358858213826e-1, 9.13545457642600895502e-1};
__device__ constexpr double kSin15[15] = {0.0, 4.06736643075800207754e-1, 7.43144825477394235015e-1, 9.51056516295153572116e-1, 9.94521895368273336923e-1, 8.66025403784438646764e-1, 5.87785252292473129169e-1, 2.07911690817759337102e-1, -2.07911690817759337102e-1, -5.87785252292473129169e-1, -8.66025403784438646764e-1, -9.94521895368273336923e-1, -9.51056516295153572116e-1, -7.43144825477394235015e-1, -4.06736643075800207754e-1};

template <typename R, int RAD, int DIR>
__device__ __forceinline__ cx_t<R> root_of_unity(int m) {
  // W_RAD^m = exp(-2 pi i DIR m / RAD)
  double c, s;
  if constexpr (RAD == 6) { c = kCos6[m]; s = kSin6[m]; }
  else if constexpr (RAD == 9) { c = kCos9[m]; s = kSin9[m]; }
  else if constexpr (RAD == 10) { c = kCos10[m]; s = kSin10[m]; }
  else if constexpr (RAD == 12) { c = kCos12[m]; s = kSin12[m]; }
  else { c = kCos15[m]; s = kSin15[m]; }
  return cx_t<R>{static_cast<R>(c), static_cast<R>(DIR > 0 ? -s : s)};
}

// (x + i y) times -i DIR: DIR (y - i x)
template <typename V, int DIR>
__device__ __forceinline__ V mul_mi(V a) {
  return DIR > 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}

// In-register DFT of RAD points (RAD = 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16), natural order in and out.
// X_k = sum_r v_r W_RAD^{r k} with W = exp(-2 pi i DIR / RAD).
template <typename R, int RAD, int DIR>
__device__ __forceinline__ void dft_reg(cx_t<R>* v) {
  using V = cx_t<R>;
  if constexpr (RAD == 6 || RAD == 9 || RAD == 10 || RAD == 12 || RAD == 15) {
    // RAD = A B: with r = a + A b and k = kb + B ka, X_k = sum_a W_A^{a ka} W_RAD^{a kb} sum_b v_{a+Ab} W_B^{b kb}
    // (B-point DFTs, twiddles, then A-point DFTs)
    constexpr int A = (RAD == 6 || RAD == 10) ? 2 : 3;
    constexpr int B = RAD / A;
    V t[RAD];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      V u[B];
#pragma unroll
      for (int b = 0; b < B; ++b) u[b] = v[a + A * b];
      dft_reg<R, B, DIR>(u);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) {
        if (a == 0 || kb == 0) {
          t[a + A * kb] = u[kb];
        } else {
          const V w = root_of_unity<R, RAD, DIR>(a * kb);
          t[a + A * kb] = V{u[kb].x * w.x - u[kb].y * w.y, u[kb].x * w.y + u[kb].y * w.x};
        }
      }
    }
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
      V w2[A];
#pragma unroll
      for (int a = 0; a < A; ++a) w2[a] = t[a + A * kb];
      dft_reg<R, A, DIR>(w2);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) v[kb + B * ka] = w2[ka];
    }
  } else if constexpr (RAD == 3) {
    // X0 = a + (b + c); X1,2 = a - (b + c)/2 -+ i DIR sin(2 pi/3) (b - c)
    const V a = v[0], b = v[1], c = v[2];
    const V t1{b.x + c.x, b.y + c.y};
    const V t2{a.x - static_cast<R>(0.5) * t1.x, a.y - static_cast<R>(0.5) * t1.y};
    const R s = static_cast<R>(kS3);
    const V t3 = mul_mi<V, DIR>(V{s * (b.x - c.x), s * (b.y - c.y)});
    v[0] = V{a.x + t1.x, a.y + t1.y};
    v[1] = V{t2.x + t3.x, t2.y + t3.y};
    v[2] = V{t2.x - t3.x, t2.y - t3.y};
  } else if constexpr (RAD == 5) {
    // pairs (b, e) and (c, d) share the real parts of W^k; their differences carry the sines
    const V a = v[0];
    const V t1{v[1].x + v[4].x, v[1].y + v[4].y}, t3{v[1].x - v[4].x, v[1].y - v[4].y};
    const V t2{v[2].x + v[3].x, v[2].y + v[3].y}, t4{v[2].x - v[3].x, v[2].y - v[3].y};
    const R c1 = static_cast<R>(kC5_1), c2 = static_cast<R>(kC5_2);
    const R s1 = static_cast<R>(kS5_1), s2 = static_cast<R>(kS5_2);
    const V m1{a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
    const V m2{a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
    const V u1 = mul_mi<V, DIR>(V{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    const V u2 = mul_mi<V, DIR>(V{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    v[0] = V{a.x + t1.x + t2.x, a.y + t1.y + t2.y};
    v[1] = V{m1.x + u1.x, m1.y + u1.y};
    v[4] = V{m1.x - u1.x, m1.y - u1.y};
    v[2] = V{m2.x + u2.x, m2.y + u2.y};
    v[3] = V{m2.x - u2.x, m2.y - u2.y};
  } else {
    // powers of two: decimation in time, iterative radix-2 with compile-time bit reversal of the input
    constexpr int LOG = RAD == 2 ? 1 : RAD == 4 ? 2 : RAD == 8 ? 3 : 4;
    V a[RAD];
#pragma unroll
    for (int i = 0; i < RAD; ++i) {
      int r = 0;
#pragma unroll
      for (int b = 0; b < LOG; ++b) r |= ((i >> b) & 1) << (LOG - 1 - b);
      a[r] = v[i];
    }
#pragma unroll
    for (int half = 1; half < RAD; half <<= 1) {
#pragma unroll
      for (int g = 0; g < RAD; g += 2 * half) {
#pragma unroll
        for (int k = 0; k < half; ++k) {
          const V w = w16<R, DIR>(k * (16 / (2 * half)));
          V t;
          const V o = a[g + k + half];
          if (k == 0) {
            t = o;
          } else {
            t.x = o.x * w.x - o.y * w.y;
            t.y = o.x * w.y + o.y * w.x;
          }
          const V e = a[g + k];
          a[g + k] = V{e.x + t.x, e.y + t.y};
          a[g + k + half] = V{e.x - t.x, e.y - t.y};
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RAD; ++i) v[i] = a[i];
  }
}

// One Stockham stage over `width` (a power of two, 2^wlog) interleaved transforms of length len; Ns is
// the product of the earlier radices, rem = len / Ns, inv_ns a float approximation of 1 / Ns used to
// split j into j div Ns and j mod Ns (exact after one correction step: j and Ns are below 2^13).
template <typename R, int RAD, int DIR, int THREADS>
__device__ __forceinline__ void fft_stage(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out, int len,
                                          int width, int wlog, int Ns, int rem, float inv_ns,
                                          const cx_t<R>* __restrict__ tw) {
  using V = cx_t<R>;
  const int nbf = len / RAD;
  const int total = nbf * width;
  const int twstep = rem / RAD;
  for (int b = threadIdx.x; b < total; b += THREADS) {
    const int j = b >> wlog;
    const int w = b & (width - 1);
    int jm = j - static_cast<int>(static_cast<float>(j) * inv_ns) * Ns;
    jm = jm < 0 ? jm + Ns : (jm >= Ns ? jm - Ns : jm);
    V v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = in[(j + r * nbf) * width + w];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        V t = tw[r * jm * twstep];
        if (DIR < 0) t.y = -t.y;
        const V o = v[r];
        v[r] = V{o.x * t.x - o.y * t.y, o.x * t.y + o.y * t.x};
      }
    }
    dft_reg<R, RAD, DIR>(v);
    const int idxD = (j - jm) * RAD + jm;
#pragma unroll
    for (int r = 0; r < RAD; ++r) out[(idxD + r * Ns) * width + w] = v[r];
  }
}

// The stage radices of a length 2^a 3^b 5^c, four bits per stage from the low end (radix 16 coded as
// 1, 0 ends the plan): 16 (if r16), 8, 4 or 2 while the remaining length is even, then 3s, then 5s.
__host__ __device__ inline uint64_t fft_radix_plan(int len, bool r16 = true) {
  uint64_t plan = 0;
  int sh = 0, rem = len;
  while (rem > 1 && sh < 64) {
    const int r = (r16 && rem % 16 == 0) ? 16 : rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 2 == 0 ? 2
                  : rem % 3 == 0 ? 3 : 5;
    plan |= static_cast<uint64_t>(r == 16 ? 1 : r) << sh;
    sh += 4;
    rem /= r;
  }
  return plan;
}

// The stage radices of a length 2^a 3^b 5^c with composite radices, fewer stages (each an LDS round
// trip): the largest of 15, 12, 10, 9, 8, 6, 5, 4, 3, 2 that divides the remaining length, four bits
// per stage from the low end (the radix itself; 0 ends the plan).
__host__ __device__ inline uint64_t fft_radix_plan_composite(int len) {
  constexpr int kRad[] = {15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  uint64_t plan = 0;
  int sh = 0, rem = len;
  while (rem > 1 && sh < 64) {
    int r = 0;
    for (int i = 0; i < 10 && r == 0; ++i)
      if (rem % kRad[i] == 0) r = kRad[i];
    if (r == 0) break;
    plan |= static_cast<uint64_t>(r) << sh;
    sh += 4;
    rem /= r;
  }
  return plan;
}

// Full transform of `width` (a power of two) interleaved length-len sequences held in A, with the
// stages of `plan` (fft_radix_plan(len, R16), or fft_radix_plan_composite(len) with COMP); B is scratch
// of the same size.  Returns the buffer holding the result.  Ends with a barrier.  Without R16 the
// radix-16 stage is not compiled in (fewer registers for kernels whose lengths are mostly odd); COMP
// compiles in the composite radices 6, 9, 10, 12 and 15.
template <typename R, int DIR, int THREADS, bool R16 = true, bool COMP = false>
__device__ cx_t<R>* lds_fft_plan(cx_t<R>* A, cx_t<R>* B, int len, int width, const cx_t<R>* __restrict__ tw,
                                 uint64_t plan) {
  using V = cx_t<R>;
  V* in = A;
  V* out = B;
  const int wlog = __builtin_ctz(static_cast<unsigned>(width));
  int Ns = 1, rem = len;
  for (; plan != 0; plan >>= 4) {
    const float inv = 1.0f / static_cast<float>(Ns);
    switch (static_cast<int>(plan & 15)) {
      case 1:
        if constexpr (R16) {
          fft_stage<R, 16, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw);
          Ns *= 16;
          rem /= 16;
        }
        break;
      case 8: fft_stage<R, 8, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 8; rem /= 8; break;
      case 4: fft_stage<R, 4, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 4; rem /= 4; break;
      case 2: fft_stage<R, 2, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 2; rem /= 2; break;
      case 3: fft_stage<R, 3, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 3; rem /= 3; break;
      case 6:
        if constexpr (COMP) { fft_stage<R, 6, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 6; rem /= 6; }
        break;
      case 9:
        if constexpr (COMP) { fft_stage<R, 9, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 9; rem /= 9; }
        break;
      case 10:
        if constexpr (COMP) { fft_stage<R, 10, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 10; rem /= 10; }
        break;
      case 12:
        if constexpr (COMP) { fft_stage<R, 12, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 12; rem /= 12; }
        break;
      case 15:
        if constexpr (COMP) { fft_stage<R, 15, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 15; rem /= 15; }
        break;
      default: fft_stage<R, 5, DIR, THREADS>(in, out, len, width, wlog, Ns, rem, inv, tw); Ns *= 5; rem /= 5; break;
    }
    __syncthreads();
    V* t = in;
    in = out;
    out = t;
  }
  return in;
}

// lds_fft_plan with the plan of len (2^a 3^b 5^c; the host checks it).
template <typename R, int DIR, int THREADS>
__device__ cx_t<R>* lds_fft(cx_t<R>* A, cx_t<R>* B, int len, int width, const cx_t<R>* __restrict__ tw) {
  return lds_fft_plan<R, DIR, THREADS>(A, B, len, width, tw, fft_radix_plan(len));
}

}  // namespace ldbp
