// Transmitter and receiver DSP on the GPU (Sec. IV-A, IV-B), built on a batched natural-order FFT.
//
//   ldbp_fft        X_k = sum_t x_t e^{-+2 pi i k t / n}, unnormalised, natural order in and out, for
//                   n = 2^a 3^b 5^c: in LDS in one pass up to 4096 samples, else column and row passes
//                   of the four-step split (tiles of a power of two of columns or rows).
//   tx_shape        16-QAM symbols -> periodic RRC-shaped waveform at rho samples/symbol:
//                   X(m) = S(m mod N_sym) H_rrc(m) sqrt(P) rho, x = IDFT(X) / n, where S is the
//                   N_sym-point DFT of the symbols (the DFT of the zero-inserted sequence is S
//                   repeated rho times).
//   rx_lpf_decimate brick-wall low-pass |f| < f_out/2 (Nyquist bin zeroed) and resampling by
//                   copying DFT bins; sample values of in-band signals are preserved.
//   rx_mse          matched filter + downsampling (the circulant M), 1/sqrt(P), genie phase
//                   phi = arg(s^H s~), per-frame MSE ||s^ - s||^2 / N_sym, and optionally the
//                   gradient of the frame-averaged MSE w.r.t. the equaliser output (phi held
//                   fixed: it minimises the loss, so its own derivative does not contribute).
//                   Downsampling by rho folds the spectrum: DFT_Nsym(s~)(m) = (1/rho) sum_b F(m + b N_sym).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "fft.h"
#include "ssm_kernels.h"
#include "txrx_kernels.h"

namespace ldbp {

constexpr int kT = 256;

template <typename V>
__device__ __forceinline__ V cmulx(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------- batched FFT

template <typename R>
__global__ void fft_twiddles(cx_t<R>* __restrict__ tab, int64_t count, int64_t mult, int64_t len) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= count) return;
  double s, c;
  sincospi(-2.0 * static_cast<double>((k * mult) % len) / static_cast<double>(len), &s, &c);
  tab[k] = cx_t<R>{static_cast<R>(c), static_cast<R>(s)};
}

template <typename R>
__global__ __launch_bounds__(kT) void fft_resident(const cx_t<R>* x, cx_t<R>* y, int n, int npol, int conj,
                                                   const cx_t<R>* __restrict__ tw) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(n) * npol;
  const int64_t off = static_cast<int64_t>(blockIdx.x) * n * npol;
  for (int e = threadIdx.x; e < n * npol; e += kT) {
    V v = x[off + e];
    if (conj) v.y = -v.y;
    A[e] = v;
  }
  __syncthreads();
  V* F = lds_fft<R, 1, kT>(A, B, n, npol, tw);
  for (int e = threadIdx.x; e < n * npol; e += kT) {
    V v = F[e];
    if (conj) v.y = -v.y;
    y[off + e] = v;
  }
}

// Column FFT over t2 of columns [c0, c0 + C) (C a power of two; columns past N1 of the last tile are
// skipped) with twiddle W_n^{t1 f2}; in -> out (same positions).
template <typename R>
__global__ __launch_bounds__(kT) void fft_col(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out, SsmGeom g,
                                              int C, int conj, const cx_t<R>* __restrict__ tw2,
                                              const cx_t<R>* __restrict__ tlo, const cx_t<R>* __restrict__ thi) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int np = g.npol, N1 = g.N1, N2 = g.N2, width = C * np;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N2) * width;
  const int nblk = (N1 + C - 1) / C;
  const int cb = static_cast<int>(blockIdx.x % static_cast<uint32_t>(nblk));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(nblk);
  const int c0 = cb * C;
  const V* iw = in + wave * g.n * np;
  V* ow = out + wave * g.n * np;
  const int tot = N2 * width;
  for (int e = threadIdx.x; e < tot; e += kT) {
    const int t2 = e / width, w = e - (e / width) * width;
    V v{0, 0};
    if (c0 + w / np < N1) {
      v = iw[(static_cast<int64_t>(t2) * N1 + c0) * np + w];
      if (conj) v.y = -v.y;
    }
    A[e] = v;
  }
  __syncthreads();
  V* F = lds_fft<R, 1, kT>(A, B, N2, width, tw2);
  for (int e = threadIdx.x; e < tot; e += kT) {
    const int f2 = e / width, w = e - (e / width) * width;
    if (c0 + w / np >= N1) continue;
    const int64_t ex = static_cast<int64_t>(c0 + w / np) * f2;
    const V t = cmulx(tlo[ex & ((int64_t(1) << g.lo_log) - 1)], thi[ex >> g.lo_log]);
    ow[(static_cast<int64_t>(f2) * N1 + c0) * np + w] = cmulx(F[e], t);
  }
}

// Row FFT over t1 of rows [f20, f20 + RW) (RW a power of two; rows past N2 of the last tile are
// skipped); result X[f2 + N2 f1] written in natural order.
template <typename R>
__global__ __launch_bounds__(kT) void fft_row(const cx_t<R>* __restrict__ in, cx_t<R>* __restrict__ out, SsmGeom g,
                                              int RW, int conj, const cx_t<R>* __restrict__ tw1) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int np = g.npol, N1 = g.N1, N2 = g.N2, width = RW * np;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N1) * width;
  const int nblk = (N2 + RW - 1) / RW;
  const int rb = static_cast<int>(blockIdx.x % static_cast<uint32_t>(nblk));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(nblk);
  const int f20 = rb * RW;
  const V* iw = in + wave * g.n * np;
  V* ow = out + wave * g.n * np;
  const int tot = N1 * width;
  for (int e = threadIdx.x; e < tot; e += kT) {
    const int r = e / (N1 * np);
    const int rem = e - r * N1 * np;
    const int t1 = rem / np, q = rem - (rem / np) * np;
    A[t1 * width + r * np + q] = f20 + r < N2 ? iw[static_cast<int64_t>(f20 + r) * N1 * np + rem] : V{0, 0};
  }
  __syncthreads();
  V* F = lds_fft<R, 1, kT>(A, B, N1, width, tw1);
  // natural order: bin k = f2 + N2 f1; for fixed f1 the RW rows are consecutive bins
  for (int e = threadIdx.x; e < tot; e += kT) {
    const int f1 = e / width, w = e - (e / width) * width;
    const int r = w / np, q = w - (w / np) * np;
    if (f20 + r >= N2) continue;
    V v = F[e];
    if (conj) v.y = -v.y;
    ow[(static_cast<int64_t>(f20 + r) + static_cast<int64_t>(N2) * f1) * np + q] = v;
  }
}

size_t fft_ws_bytes(int dtype, int64_t nwave, int64_t n, int npol) {
  const SsmGeom g = make_geom(dtype, nwave, n, npol, 1.0, 0.0, 0.0);
  size_t tab = g.resident ? static_cast<size_t>(n)
                          : static_cast<size_t>(g.N1) + g.N2 + (int64_t(1) << g.lo_log) + (n >> g.lo_log) + 1;
  size_t b = ((tab * cx_size(dtype)) + 255) & ~size_t(255);
  if (!g.resident) b += static_cast<size_t>(nwave) * n * npol * cx_size(dtype);
  return b;
}

static int fft_tile(int dtype, const SsmGeom& g) {
  const int64_t total = g.n * g.npol * g.nwave;
  int e = dtype == LDBP_C64 ? 4096 : 2048;
  while (e > 512 && total / e < 2048) e /= 2;
  return e;
}

// largest power of two <= max(1, v), capped at the power of two >= cap
static int tile_pow2(int64_t v, int64_t cap) {
  int p = 1;
  while (2 * static_cast<int64_t>(p) <= v && p < cap) p *= 2;
  return p;
}

// columns per column tile and rows per row tile of the four-step transform (powers of two)
static void fft_tiles(int dtype, const SsmGeom& g, int& C, int& RW) {
  const int E = fft_tile(dtype, g);
  C = tile_pow2(E / (static_cast<int64_t>(g.N2) * g.npol), g.N1);
  RW = tile_pow2(E / (static_cast<int64_t>(g.N1) * g.npol), g.N2);
}

size_t fft_lds_bytes(int dtype, int64_t nwave, int64_t n, int npol) {
  const SsmGeom g = make_geom(dtype, nwave, n, npol, 1.0, 0.0, 0.0);
  if (g.resident) return 2 * static_cast<size_t>(n) * npol * cx_size(dtype);
  int C, RW;
  fft_tiles(dtype, g, C, RW);
  return 2 * std::max(static_cast<size_t>(g.N2) * C, static_cast<size_t>(g.N1) * RW) * npol * cx_size(dtype);
}

template <typename R>
static int fft_run_t(int64_t nwave, int64_t n, int npol, const void* x, void* y, int inverse, void* ws,
                     hipStream_t s) {
  using V = cx_t<R>;
  const int dtype = sizeof(R) == 4 ? LDBP_C64 : LDBP_C128;
  const SsmGeom g = make_geom(dtype, nwave, n, npol, 1.0, 0.0, 0.0);
  V* tab = static_cast<V*>(ws);
  auto gen = [&](V* dst, int64_t count, int64_t mult, int64_t len) -> int {
    hipLaunchKernelGGL(fft_twiddles<R>, dim3(static_cast<uint32_t>((count + 255) / 256)), dim3(256), 0, s, dst,
                       count, mult, len);
    LDBP_HIP_CHECK(hipGetLastError());
    return LDBP_OK;
  };
  if (g.resident) {
    int st = gen(tab, n, 1, n);
    if (st) return st;
    const size_t lds = 2 * static_cast<size_t>(n) * npol * sizeof(V);
    if (lds > 65536)
      LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fft_resident<R>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(fft_resident<R>, dim3(static_cast<uint32_t>(nwave)), dim3(kT), lds, s,
                       static_cast<const V*>(x), static_cast<V*>(y), static_cast<int>(n), npol, inverse, tab);
    LDBP_HIP_CHECK(hipGetLastError());
    return LDBP_OK;
  }
  V* tw1 = tab;
  V* tw2 = tw1 + g.N1;
  V* tlo = tw2 + g.N2;
  V* thi = tlo + (int64_t(1) << g.lo_log);
  const size_t tabb = ((static_cast<size_t>(g.N1) + g.N2 + (int64_t(1) << g.lo_log) + (n >> g.lo_log) + 1) *
                       sizeof(V) + 255) & ~size_t(255);
  V* tmp = reinterpret_cast<V*>(static_cast<char*>(ws) + tabb);
  const int64_t lo = int64_t(1) << g.lo_log;
  int st = gen(tw1, g.N1, 1, g.N1);
  if (!st) st = gen(tw2, g.N2, 1, g.N2);
  if (!st) st = gen(tlo, lo, 1, n);
  if (!st) st = gen(thi, (n + lo - 1) / lo, lo, n);
  if (st) return st;
  int C, RW;
  fft_tiles(dtype, g, C, RW);
  const size_t lc = 2 * static_cast<size_t>(g.N2) * C * npol * sizeof(V);
  const size_t lr = 2 * static_cast<size_t>(g.N1) * RW * npol * sizeof(V);
  if (lc > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fft_col<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lc)));
  if (lr > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fft_row<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lr)));
  hipLaunchKernelGGL(fft_col<R>, dim3(static_cast<uint32_t>(((g.N1 + C - 1) / C) * nwave)), dim3(kT), lc, s,
                     static_cast<const V*>(x), tmp, g, C, inverse, tw2, tlo, thi);
  LDBP_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(fft_row<R>, dim3(static_cast<uint32_t>(((g.N2 + RW - 1) / RW) * nwave)), dim3(kT), lr, s, tmp,
                     static_cast<V*>(y), g, RW, inverse, tw1);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

int fft_run(int dtype, int64_t nwave, int64_t n, int npol, const void* x, void* y, int inverse, void* ws,
            hipStream_t s) {
  return dtype == LDBP_C64 ? fft_run_t<float>(nwave, n, npol, x, y, inverse, ws, s)
                           : fft_run_t<double>(nwave, n, npol, x, y, inverse, ws, s);
}

// ---------------------------------------------------------------- spectral helpers

// Root-raised-cosine response (unit passband) at frequency |f| (Hz).
__device__ __forceinline__ double rrc_h(double f, double rs, double beta) {
  f = fabs(f);
  const double f1 = (1.0 - beta) * rs / 2.0, f2 = (1.0 + beta) * rs / 2.0;
  if (f <= f1) return 1.0;
  if (f > f2) return 0.0;
  return sqrt(0.5 * (1.0 + cos(M_PI / (beta * rs) * (f - f1))));
}

// signed DFT frequency index of bin k on an n-point grid (Nyquist bin negative)
__device__ __forceinline__ int64_t sbin(int64_t k, int64_t n) { return k < (n + 1) / 2 ? k : k - n; }

// 16-QAM symbols from indices: (2 (i mod 4) - 3 + j (2 (i div 4) - 3)) / sqrt(10)
template <typename R>
__global__ void qam16_map(const int32_t* __restrict__ idx, cx_t<R>* __restrict__ s, int64_t count) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= count) return;
  const int i = idx[e] & 15;
  const R sc = static_cast<R>(0.31622776601683793320);
  s[e] = cx_t<R>{static_cast<R>(2 * (i & 3) - 3) * sc, static_cast<R>(2 * (i >> 2) - 3) * sc};
}

// X(m) = S(m mod nsym) H_rrc(m) sqrt(P_w) rho / n  for m < n (then an inverse DFT gives the waveform)
template <typename R>
__global__ void tx_spectrum(const cx_t<R>* __restrict__ S, cx_t<R>* __restrict__ X, int64_t nwave, int64_t nsym,
                            int64_t n, int npol, double fs, double rs, double beta, const double* __restrict__ p,
                            int rho) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t per = n * npol;
  if (e >= nwave * per) return;
  const int64_t w = e / per, r = e - w * per;
  const int64_t m = r / npol;
  const int q = static_cast<int>(r - m * npol);
  const double h = rrc_h(static_cast<double>(sbin(m, n)) * fs / static_cast<double>(n), rs, beta);
  const double gain = h * sqrt(p[w]) * rho / static_cast<double>(n);
  const cx_t<R> v = S[(w * nsym + (m % nsym)) * npol + q];
  X[e] = cx_t<R>{static_cast<R>(v.x * gain), static_cast<R>(v.y * gain)};
}

// Z (n_out bins) from Y (n_in bins): |f| < f_out/2 kept, Nyquist bin zero, scaled by 1/n_in
// (resampling scale n_out/n_in times the inverse-DFT normalisation 1/n_out).
template <typename R>
__global__ void lpf_bins(const cx_t<R>* __restrict__ Y, cx_t<R>* __restrict__ Z, int64_t nwave, int64_t nin,
                         int64_t nout, int npol) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t per = nout * npol;
  if (e >= nwave * per) return;
  const int64_t w = e / per, r = e - w * per;
  const int64_t m = r / npol;
  const int q = static_cast<int>(r - m * npol);
  const int64_t h = nout / 2;
  cx_t<R> v{0, 0};
  if (m != h) {
    const int64_t src = m < h ? m : m - nout + nin;
    v = Y[(w * nin + src) * npol + q];
    const R sc = static_cast<R>(1.0 / static_cast<double>(nin));
    v.x *= sc;
    v.y *= sc;
  }
  Z[e] = v;
}

// fold(m) = sum_b Z(m + b nsym) H_rrc(m + b nsym) / (n sqrt(P))  (n = rho nsym bins)
template <typename R>
__global__ void mf_fold(const cx_t<R>* __restrict__ Z, cx_t<R>* __restrict__ Fo, int64_t nwave, int64_t nsym,
                        int npol, int rho, double fs, double rs, double beta, const double* __restrict__ p) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t per = nsym * npol;
  if (e >= nwave * per) return;
  const int64_t w = e / per, r = e - w * per;
  const int64_t m = r / npol;
  const int q = static_cast<int>(r - m * npol);
  const int64_t n = nsym * rho;
  double ax = 0, ay = 0;
  for (int b = 0; b < rho; ++b) {
    const int64_t k = m + b * nsym;
    const double h = rrc_h(static_cast<double>(sbin(k, n)) * fs / static_cast<double>(n), rs, beta);
    const cx_t<R> v = Z[(w * n + k) * npol + q];
    ax += h * v.x;
    ay += h * v.y;
  }
  const double sc = 1.0 / (static_cast<double>(n) * sqrt(p[w]));
  Fo[e] = cx_t<R>{static_cast<R>(ax * sc), static_cast<R>(ay * sc)};
}

// Per frame (and polarisation): phi = arg(sum conj(s) s~), s^ = s~ e^{-j phi}, mse = mean |s^ - s|^2,
// and G_s~ = e^{j phi} 2 (s^ - s) / (nsym * nframes) when grad is requested.  One workgroup per frame.
template <typename R>
__global__ __launch_bounds__(kT) void phase_mse(const cx_t<R>* __restrict__ st, const cx_t<R>* __restrict__ s,
                                                int64_t nsym, int npol, int64_t nframes, cx_t<R>* __restrict__ shat,
                                                double* __restrict__ mse, cx_t<R>* __restrict__ gst) {
  __shared__ double rx[kT], ry[kT];
  const int64_t f = blockIdx.x;  // frame = wave * npol + pol
  const int64_t w = f / npol;
  const int q = static_cast<int>(f - w * npol);
  auto at = [&](int64_t k) { return (w * nsym + k) * npol + q; };
  double ax = 0, ay = 0;
  for (int64_t k = threadIdx.x; k < nsym; k += kT) {
    const cx_t<R> a = s[at(k)], b = st[at(k)];
    ax += static_cast<double>(a.x) * b.x + static_cast<double>(a.y) * b.y;
    ay += static_cast<double>(a.x) * b.y - static_cast<double>(a.y) * b.x;
  }
  rx[threadIdx.x] = ax;
  ry[threadIdx.x] = ay;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o) {
      rx[threadIdx.x] += rx[threadIdx.x + o];
      ry[threadIdx.x] += ry[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double phi = atan2(ry[0], rx[0]);
  __syncthreads();
  double sn, cs;
  sincos(phi, &sn, &cs);
  const double gsc = 2.0 / (static_cast<double>(nsym) * nframes);
  double err = 0;
  for (int64_t k = threadIdx.x; k < nsym; k += kT) {
    const cx_t<R> b = st[at(k)], a = s[at(k)];
    const double hx = b.x * cs + b.y * sn, hy = b.y * cs - b.x * sn;  // s~ e^{-j phi}
    const double dx = hx - a.x, dy = hy - a.y;
    err += dx * dx + dy * dy;
    if (shat) shat[at(k)] = cx_t<R>{static_cast<R>(hx), static_cast<R>(hy)};
    if (gst) {
      const double gx = gsc * dx, gy = gsc * dy;  // e^{+j phi} G_s^
      gst[at(k)] = cx_t<R>{static_cast<R>(gx * cs - gy * sn), static_cast<R>(gx * sn + gy * cs)};
    }
  }
  rx[threadIdx.x] = err;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (static_cast<int>(threadIdx.x) < o) rx[threadIdx.x] += rx[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) mse[f] = rx[0] / static_cast<double>(nsym);
}

// G(m) = H_rrc(m) Gs(m mod nsym) / (n sqrt(P)) for m < n = rho nsym (adjoint of fold)
template <typename R>
__global__ void mf_unfold(const cx_t<R>* __restrict__ Gs, cx_t<R>* __restrict__ Gz, int64_t nwave, int64_t nsym,
                          int npol, int rho, double fs, double rs, double beta, const double* __restrict__ p) {
  const int64_t n = nsym * rho;
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t per = n * npol;
  if (e >= nwave * per) return;
  const int64_t w = e / per, r = e - w * per;
  const int64_t k = r / npol;
  const int q = static_cast<int>(r - k * npol);
  const double h = rrc_h(static_cast<double>(sbin(k, n)) * fs / static_cast<double>(n), rs, beta);
  const double sc = h / (static_cast<double>(n) * sqrt(p[w]));
  const cx_t<R> v = Gs[(w * nsym + (k % nsym)) * npol + q];
  Gz[e] = cx_t<R>{static_cast<R>(v.x * sc), static_cast<R>(v.y * sc)};
}

static uint32_t blocks_for(int64_t count) { return static_cast<uint32_t>((count + kT - 1) / kT); }

// Symbols from 16-QAM indices (idx) or given directly (sym, complex [nwave][nsym][npol]; idx NULL).
template <typename R>
int tx_run_t(int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const int32_t* idx,
             const double* p, void* x, char* ws, hipStream_t s, const void* sym) {
  using V = cx_t<R>;
  const int dtype = sizeof(R) == 4 ? LDBP_C64 : LDBP_C128;
  const int64_t n = nsym * rho;
  V* S = reinterpret_cast<V*>(ws);
  const size_t sb = (static_cast<size_t>(nwave) * nsym * npol * sizeof(V) + 255) & ~size_t(255);
  V* X = reinterpret_cast<V*>(ws + sb);
  const size_t xb = (static_cast<size_t>(nwave) * n * npol * sizeof(V) + 255) & ~size_t(255);
  char* fws = ws + sb + xb;
  const int64_t cs = nwave * nsym * npol;
  const V* src = S;
  if (sym) {
    src = static_cast<const V*>(sym);
  } else {
    hipLaunchKernelGGL(qam16_map<R>, dim3(blocks_for(cs)), dim3(kT), 0, s, idx, S, cs);
    LDBP_HIP_CHECK(hipGetLastError());
  }
  int st = fft_run(dtype, nwave, nsym, npol, src, S, 0, fws, s);
  if (st) return st;
  const int64_t cx = nwave * n * npol;
  hipLaunchKernelGGL(tx_spectrum<R>, dim3(blocks_for(cx)), dim3(kT), 0, s, S, X, nwave, nsym, n, npol,
                     rho * rs, rs, beta, p, rho);
  LDBP_HIP_CHECK(hipGetLastError());
  return fft_run(dtype, nwave, n, npol, X, x, 1, fws, s);
}

size_t tx_ws_bytes(int dtype, int64_t nwave, int64_t nsym, int npol, int rho) {
  const int64_t n = nsym * rho;
  const size_t sb = (static_cast<size_t>(nwave) * nsym * npol * cx_size(dtype) + 255) & ~size_t(255);
  const size_t xb = (static_cast<size_t>(nwave) * n * npol * cx_size(dtype) + 255) & ~size_t(255);
  return sb + xb + std::max(fft_ws_bytes(dtype, nwave, nsym, npol), fft_ws_bytes(dtype, nwave, n, npol));
}

int tx_run(int dtype, int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const int32_t* idx,
           const double* p, void* x, void* ws, hipStream_t s, const void* sym) {
  return dtype == LDBP_C64
             ? tx_run_t<float>(nwave, nsym, npol, rho, rs, beta, idx, p, x, static_cast<char*>(ws), s, sym)
             : tx_run_t<double>(nwave, nsym, npol, rho, rs, beta, idx, p, x, static_cast<char*>(ws), s, sym);
}

size_t lpf_ws_bytes(int dtype, int64_t nwave, int64_t nin, int64_t nout, int npol) {
  const size_t yb = (static_cast<size_t>(nwave) * nin * npol * cx_size(dtype) + 255) & ~size_t(255);
  const size_t zb = (static_cast<size_t>(nwave) * nout * npol * cx_size(dtype) + 255) & ~size_t(255);
  return yb + zb + std::max(fft_ws_bytes(dtype, nwave, nin, npol), fft_ws_bytes(dtype, nwave, nout, npol));
}

int lpf_run(int dtype, int64_t nwave, int64_t nin, int64_t nout, int npol, const void* y, void* r, void* ws,
            hipStream_t s) {
  char* b = static_cast<char*>(ws);
  const size_t yb = (static_cast<size_t>(nwave) * nin * npol * cx_size(dtype) + 255) & ~size_t(255);
  const size_t zb = (static_cast<size_t>(nwave) * nout * npol * cx_size(dtype) + 255) & ~size_t(255);
  void* Y = b;
  void* Z = b + yb;
  char* fws = b + yb + zb;
  int st = fft_run(dtype, nwave, nin, npol, y, Y, 0, fws, s);
  if (st) return st;
  const int64_t cnt = nwave * nout * npol;
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(lpf_bins<float>, dim3(blocks_for(cnt)), dim3(kT), 0, s, static_cast<const float2*>(Y),
                       static_cast<float2*>(Z), nwave, nin, nout, npol);
  else
    hipLaunchKernelGGL(lpf_bins<double>, dim3(blocks_for(cnt)), dim3(kT), 0, s, static_cast<const double2*>(Y),
                       static_cast<double2*>(Z), nwave, nin, nout, npol);
  LDBP_HIP_CHECK(hipGetLastError());
  return fft_run(dtype, nwave, nout, npol, Z, r, 1, fws, s);
}

size_t rx_ws_bytes(int dtype, int64_t nwave, int64_t nsym, int npol, int rho) {
  const int64_t n = nsym * rho;
  const size_t zb = (static_cast<size_t>(nwave) * n * npol * cx_size(dtype) + 255) & ~size_t(255);
  const size_t sb = (static_cast<size_t>(nwave) * nsym * npol * cx_size(dtype) + 255) & ~size_t(255);
  return 2 * zb + 2 * sb + std::max(fft_ws_bytes(dtype, nwave, n, npol), fft_ws_bytes(dtype, nwave, nsym, npol));
}

template <typename R>
int rx_run_t(int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const void* z, const void* sym,
             const double* p, void* shat, double* mse, void* gz, char* ws, hipStream_t s) {
  using V = cx_t<R>;
  const int dtype = sizeof(R) == 4 ? LDBP_C64 : LDBP_C128;
  const int64_t n = nsym * rho;
  const size_t zb = (static_cast<size_t>(nwave) * n * npol * sizeof(V) + 255) & ~size_t(255);
  const size_t sb = (static_cast<size_t>(nwave) * nsym * npol * sizeof(V) + 255) & ~size_t(255);
  V* Z = reinterpret_cast<V*>(ws);
  V* Z2 = reinterpret_cast<V*>(ws + zb);
  V* Fo = reinterpret_cast<V*>(ws + 2 * zb);
  V* G = reinterpret_cast<V*>(ws + 2 * zb + sb);
  char* fws = ws + 2 * zb + 2 * sb;
  const double fs = rho * rs;
  int st = fft_run(dtype, nwave, n, npol, z, Z, 0, fws, s);
  if (st) return st;
  const int64_t cs = nwave * nsym * npol;
  hipLaunchKernelGGL(mf_fold<R>, dim3(blocks_for(cs)), dim3(kT), 0, s, Z, Fo, nwave, nsym, npol, rho, fs, rs, beta,
                     p);
  LDBP_HIP_CHECK(hipGetLastError());
  st = fft_run(dtype, nwave, nsym, npol, Fo, Fo, 1, fws, s);  // s~ (unnormalised inverse; scale applied in fold)
  if (st) return st;
  hipLaunchKernelGGL(phase_mse<R>, dim3(static_cast<uint32_t>(nwave * npol)), dim3(kT), 0, s, Fo,
                     static_cast<const V*>(sym), nsym, npol, nwave * npol, static_cast<V*>(shat), mse,
                     gz ? G : nullptr);
  LDBP_HIP_CHECK(hipGetLastError());
  if (!gz) return LDBP_OK;
  st = fft_run(dtype, nwave, nsym, npol, G, G, 0, fws, s);
  if (st) return st;
  const int64_t cz = nwave * n * npol;
  hipLaunchKernelGGL(mf_unfold<R>, dim3(blocks_for(cz)), dim3(kT), 0, s, G, Z2, nwave, nsym, npol, rho, fs, rs,
                     beta, p);
  LDBP_HIP_CHECK(hipGetLastError());
  return fft_run(dtype, nwave, n, npol, Z2, gz, 1, fws, s);
}

int rx_run(int dtype, int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const void* z,
           const void* sym, const double* p, void* shat, double* mse, void* gz, void* ws, hipStream_t s) {
  return dtype == LDBP_C64
             ? rx_run_t<float>(nwave, nsym, npol, rho, rs, beta, z, sym, p, shat, mse, gz, static_cast<char*>(ws), s)
             : rx_run_t<double>(nwave, nsym, npol, rho, rs, beta, z, sym, p, shat, mse, gz, static_cast<char*>(ws),
                                s);
}

int qam_run(int dtype, int64_t count, const int32_t* idx, void* s, hipStream_t st) {
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(qam16_map<float>, dim3(blocks_for(count)), dim3(kT), 0, st, idx, static_cast<float2*>(s), count);
  else
    hipLaunchKernelGGL(qam16_map<double>, dim3(blocks_for(count)), dim3(kT), 0, st, idx, static_cast<double2*>(s),
                       count);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

}  // namespace ldbp
