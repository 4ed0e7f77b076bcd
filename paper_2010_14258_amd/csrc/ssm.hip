// Split-step engine: the FFT-based channel simulator and FFT digital backpropagation
// (Sec. III-A: time-discretised NLSE; Sec. IV-A: spans, amplifiers).
//
// Both are programs of the form  P_0, L_1, P_1, L_2, ..., L_M, P_M  where
//   L_i  is a linear step X_k <- X_k exp(z_i (j beta2 w_k^2 / 2 - alpha / 2)) in the DFT domain
//        (z_i < 0 for backpropagation), and
//   P_i  is a pointwise operation: Kerr phase (ka), gain g, additive noise sigma * w (from a
//        noise buffer slot), Kerr phase (kb), in that order, where a Kerr phase with
//        coefficient k rotates a sample by k (|x|^2 summed over polarisations).
// The C ABI (api_ssm.hip) turns a link description into such a program.
//
// Execution paths
//   resident  n <= 4096: one workgroup per waveform keeps the waveform in LDS for the whole
//             program (forward FFT, response, inverse FFT, pointwise op per step).
//   four-step n = N1 N2 > 4096: position t = t1 + N1 t2, frequency k = f2 + N2 f1.
//     column pass (per group of columns t1): inverse column FFT over f2 of the previous step,
//       P_i, forward column FFT over t2, twiddle W_n^{t1 f2};
//     row pass (per group of rows f2): forward row FFT over t1 -> f1 (bin k = f2 + N2 f1),
//       multiply by the step response and 1/n, inverse row FFT, twiddle W_n^{-t1 f2}.
//   So a step costs one read and one write of the waveform in each of two passes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "fft.h"
#include "ssm_kernels.h"

namespace ldbp {

constexpr int kSsmThreads = 256;

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

template <typename V>
__device__ __forceinline__ V cmul_t(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------- twiddle tables

// tab[k] = exp(-2 pi i k * mult / len) for k < count, computed in FP64.
template <typename R>
__global__ void twiddle_table(cx_t<R>* __restrict__ tab, int64_t count, int64_t mult, int64_t len) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= count) return;
  const int64_t e = (k * mult) % len;
  double s, c;
  sincospi(-2.0 * static_cast<double>(e) / static_cast<double>(len), &s, &c);
  tab[k] = cx_t<R>{static_cast<R>(c), static_cast<R>(s)};
}

template <typename R>
__device__ __forceinline__ cx_t<R> twiddle_n(int64_t e, int lo_log, const cx_t<R>* __restrict__ tlo,
                                             const cx_t<R>* __restrict__ thi) {
  const cx_t<R> a = tlo[e & ((1 << lo_log) - 1)];
  const cx_t<R> b = thi[e >> lo_log];
  return cmul_t(a, b);
}

// ---------------------------------------------------------------- resident path

template <typename R>
__global__ __launch_bounds__(kSsmThreads) void ssm_resident_kernel(const cx_t<R>* x, cx_t<R>* y, SsmGeom g,
                                                                   const double* __restrict__ lin_z,
                                                                   const PwOp* __restrict__ ops, int32_t M,
                                                                   const cx_t<R>* __restrict__ noise,
                                                                   const cx_t<R>* __restrict__ tw) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = static_cast<int>(g.n);
  const int np = g.npol;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(n) * np;
  const int64_t wave = blockIdx.x;
  const V* xw = x + wave * g.n * np;
  V* yw = y + wave * g.n * np;
  for (int e = threadIdx.x; e < n * np; e += kSsmThreads) A[e] = xw[e];
  __syncthreads();
  const R inv_n = static_cast<R>(1.0 / static_cast<double>(n));
  for (int i = 0; i <= M; ++i) {
    const PwOp op = ops[i];
    const V* nz = (op.slot >= 0 && noise) ? noise + (static_cast<int64_t>(op.slot) * g.nwave + wave) * g.n * np
                                           : nullptr;
    for (int t = threadIdx.x; t < n; t += kSsmThreads) {
      V v[2];
      for (int q = 0; q < np; ++q) v[q] = A[t * np + q];
      apply_pw<R>(v, np, op, nz ? nz + static_cast<int64_t>(t) * np : nullptr);
      for (int q = 0; q < np; ++q) A[t * np + q] = v[q];
    }
    __syncthreads();
    if (i == M) break;
    V* F = lds_fft<R, 1, kSsmThreads>(A, B, n, np, tw);
    V* other = (F == A) ? B : A;
    const double z = lin_z[i];
    const double zrev = z * g.beta2 * M_PI * g.fs * g.fs / (static_cast<double>(n) * n);
    const R amp = static_cast<R>(exp(-0.5 * z * g.alpha)) * inv_n;
    for (int e = threadIdx.x; e < n * np; e += kSsmThreads) {
      const int k = e / np;
      F[e] = cmul_t(F[e], lin_response<R>(k, n, zrev, amp));
    }
    __syncthreads();
    V* T = lds_fft<R, -1, kSsmThreads>(F, other, n, np, tw);
    if (T != A) {
      for (int e = threadIdx.x; e < n * np; e += kSsmThreads) A[e] = T[e];
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < n * np; e += kSsmThreads) yw[e] = A[e];
}

// ---------------------------------------------------------------- four-step passes

// Column pass over columns [cb*C, cb*C + C) of one waveform (LDS [N2][C*npol]).
template <typename R>
__global__ __launch_bounds__(kSsmThreads) void ssm_col_kernel(const cx_t<R>* src, cx_t<R>* dst, SsmGeom g,
                                                              int32_t C,
                                                              const PwOp* __restrict__ ops, int32_t op_index,
                                                              int32_t do_ifft, int32_t do_fft,
                                                              const cx_t<R>* __restrict__ noise,
                                                              const cx_t<R>* __restrict__ tw2,
                                                              const cx_t<R>* __restrict__ tlo,
                                                              const cx_t<R>* __restrict__ thi) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int np = g.npol;
  const int N1 = g.N1, N2 = g.N2;
  const int width = C * np;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N2) * width;
  const int nblk = N1 / C;
  const int cb = static_cast<int>(blockIdx.x % static_cast<uint32_t>(nblk));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(nblk);
  const int c0 = cb * C;
  const V* sw = src + wave * g.n * np;
  V* dw = dst + wave * g.n * np;
  const int tot = N2 * width;
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int t2 = e / width;
    const int w = e - t2 * width;
    A[e] = sw[(static_cast<int64_t>(t2) * N1 + c0) * np + w];
  }
  __syncthreads();
  V* cur = A;
  if (do_ifft) cur = lds_fft<R, -1, kSsmThreads>(A, B, N2, width, tw2);
  V* other = (cur == A) ? B : A;
  const PwOp op = ops[op_index];
  const V* nz = (op.slot >= 0 && noise) ? noise + (static_cast<int64_t>(op.slot) * g.nwave + wave) * g.n * np
                                         : nullptr;
  for (int e = threadIdx.x; e < N2 * C; e += kSsmThreads) {
    const int t2 = e / C;
    const int c = e - t2 * C;
    V v[2];
    for (int q = 0; q < np; ++q) v[q] = cur[t2 * width + c * np + q];
    apply_pw<R>(v, np, op, nz ? nz + (static_cast<int64_t>(t2) * N1 + c0 + c) * np : nullptr);
    for (int q = 0; q < np; ++q) cur[t2 * width + c * np + q] = v[q];
  }
  __syncthreads();
  if (do_fft) {
    cur = lds_fft<R, 1, kSsmThreads>(cur, other, N2, width, tw2);
    for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
      const int f2 = e / width;
      const int w = e - f2 * width;
      const int t1 = c0 + w / np;
      cur[e] = cmul_t(cur[e], twiddle_n<R>(static_cast<int64_t>(t1) * f2, g.lo_log, tlo, thi));
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int t2 = e / width;
    const int w = e - t2 * width;
    dw[(static_cast<int64_t>(t2) * N1 + c0) * np + w] = cur[e];
  }
}

// Row pass over rows [rb*RW, rb*RW + RW) (LDS transposed to [N1][RW*npol]).
template <typename R>
__global__ __launch_bounds__(kSsmThreads) void ssm_row_kernel(cx_t<R>* __restrict__ data, SsmGeom g, int32_t RW,
                                                              double z, const cx_t<R>* __restrict__ tw1,
                                                              const cx_t<R>* __restrict__ tlo,
                                                              const cx_t<R>* __restrict__ thi) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int np = g.npol;
  const int N1 = g.N1, N2 = g.N2;
  const int width = RW * np;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N1) * width;
  const int nblk = N2 / RW;
  const int rb = static_cast<int>(blockIdx.x % static_cast<uint32_t>(nblk));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(nblk);
  const int f20 = rb * RW;
  V* dw = data + wave * g.n * np;
  const int tot = N1 * width;
  // global row f2 = f20 + r holds N1*np contiguous values; LDS element (t1, r*np + q)
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int r = e / (N1 * np);
    const int rem = e - r * N1 * np;
    const int t1 = rem / np;
    const int q = rem - t1 * np;
    A[t1 * width + r * np + q] = dw[static_cast<int64_t>(f20 + r) * N1 * np + rem];
  }
  __syncthreads();
  V* F = lds_fft<R, 1, kSsmThreads>(A, B, N1, width, tw1);
  V* other = (F == A) ? B : A;
  const double zrev = z * g.beta2 * M_PI * g.fs * g.fs / (static_cast<double>(g.n) * g.n);
  const R amp = static_cast<R>(exp(-0.5 * z * g.alpha) / static_cast<double>(g.n));
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int f1 = e / width;
    const int r = (e - f1 * width) / np;
    const int64_t k = static_cast<int64_t>(f20 + r) + static_cast<int64_t>(N2) * f1;
    F[e] = cmul_t(F[e], lin_response<R>(k, g.n, zrev, amp));
  }
  __syncthreads();
  V* T = lds_fft<R, -1, kSsmThreads>(F, other, N1, width, tw1);
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int t1 = e / width;
    const int r = (e - t1 * width) / np;
    V w = twiddle_n<R>(static_cast<int64_t>(t1) * (f20 + r), g.lo_log, tlo, thi);
    w.y = -w.y;
    T[e] = cmul_t(T[e], w);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < tot; e += kSsmThreads) {
    const int r = e / (N1 * np);
    const int rem = e - r * N1 * np;
    const int t1 = rem / np;
    const int q = rem - t1 * np;
    dw[static_cast<int64_t>(f20 + r) * N1 * np + rem] = T[t1 * width + r * np + q];
  }
}

// ---------------------------------------------------------------- host side

static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

SsmGeom make_geom(int dtype, int64_t nwave, int64_t n, int npol, double fs, double alpha, double beta2) {
  SsmGeom g{};
  g.n = n;
  g.nwave = nwave;
  g.npol = npol;
  g.fs = fs;
  g.alpha = alpha;
  g.beta2 = beta2;
  if (n <= kSsmResidentMax && 2 * n * npol * static_cast<int64_t>(cx_size(dtype)) <= 128 * 1024) {
    g.resident = 1;
    g.N1 = static_cast<int32_t>(n);
    g.N2 = 1;
  } else {
    g.resident = 0;
    int64_t N2 = n >= (int64_t(1) << 16) ? 256 : n / 256;
    if (n / N2 > 4096) N2 = n / 4096;
    g.N2 = static_cast<int32_t>(N2);
    g.N1 = static_cast<int32_t>(n / N2);
  }
  g.lo_log = (ilog2(n) + 1) / 2;
  return g;
}

size_t ssm_table_elems(const SsmGeom& g) {
  if (g.resident) return static_cast<size_t>(g.n);
  return static_cast<size_t>(g.N1) + g.N2 + (int64_t(1) << g.lo_log) + (g.n >> g.lo_log) + 1;
}

static size_t elem_size(int dtype) { return cx_size(dtype); }

// elements per workgroup tile of the four-step passes
static int tile_elems(int dtype, const SsmGeom& g) {
  const int64_t total = g.n * g.npol * g.nwave;
  int e = dtype == LDBP_C64 ? 4096 : 2048;
  while (e > 512 && total / e < 2048) e /= 2;
  return e;
}

template <typename R>
static int run_t(const SsmGeom& g, const void* x, void* y, const double* lin_z_dev, const void* ops_dev, int32_t M,
                 const std::vector<double>& lin_z_host, const void* noise, void* tables, hipStream_t s) {
  using V = cx_t<R>;
  V* tab = static_cast<V*>(tables);
  auto gen = [&](V* dst, int64_t count, int64_t mult, int64_t len) -> int {
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(twiddle_table<R>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, dst, count, mult,
                       len);
    LDBP_HIP_CHECK(hipGetLastError());
    return LDBP_OK;
  };
  const int dtype = sizeof(R) == 4 ? LDBP_C64 : LDBP_C128;
  if (g.resident) {
    int st = gen(tab, g.n, 1, g.n);
    if (st) return st;
    const size_t lds = 2 * static_cast<size_t>(g.n) * g.npol * sizeof(V);
    auto kern = ssm_resident_kernel<R>;
    if (lds > 65536)
      LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(g.nwave)), dim3(kSsmThreads), lds, s,
                       static_cast<const V*>(x), static_cast<V*>(y), g, lin_z_dev,
                       static_cast<const PwOp*>(ops_dev), M, static_cast<const V*>(noise), tab);
    LDBP_HIP_CHECK(hipGetLastError());
    return LDBP_OK;
  }
  V* tw1 = tab;
  V* tw2 = tw1 + g.N1;
  V* tlo = tw2 + g.N2;
  V* thi = tlo + (int64_t(1) << g.lo_log);
  int st = gen(tw1, g.N1, 1, g.N1);
  if (!st) st = gen(tw2, g.N2, 1, g.N2);
  if (!st) st = gen(tlo, int64_t(1) << g.lo_log, 1, g.n);
  if (!st) st = gen(thi, (g.n >> g.lo_log), int64_t(1) << g.lo_log, g.n);
  if (st) return st;
  const int E = tile_elems(dtype, g);
  const int C = std::max(1, std::min<int>(g.N1, E / (g.N2 * g.npol)));
  const int RW = std::max(1, std::min<int>(g.N2, E / (g.N1 * g.npol)));
  const size_t lds_c = 2 * static_cast<size_t>(g.N2) * C * g.npol * sizeof(V);
  const size_t lds_r = 2 * static_cast<size_t>(g.N1) * RW * g.npol * sizeof(V);
  auto kc = ssm_col_kernel<R>;
  auto kr = ssm_row_kernel<R>;
  if (lds_c > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kc), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_c)));
  if (lds_r > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kr), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_r)));
  const uint32_t gc = static_cast<uint32_t>((g.N1 / C) * g.nwave);
  const uint32_t gr = static_cast<uint32_t>((g.N2 / RW) * g.nwave);
  const V* nz = static_cast<const V*>(noise);
  for (int i = 0; i <= M; ++i) {
    const V* src = (i == 0) ? static_cast<const V*>(x) : static_cast<const V*>(y);
    hipLaunchKernelGGL(kc, dim3(gc), dim3(kSsmThreads), lds_c, s, src, static_cast<V*>(y), g, C,
                       static_cast<const PwOp*>(ops_dev), i, i > 0 ? 1 : 0, i < M ? 1 : 0, nz, tw2, tlo, thi);
    LDBP_HIP_CHECK(hipGetLastError());
    if (i == M) break;
    hipLaunchKernelGGL(kr, dim3(gr), dim3(kSsmThreads), lds_r, s, static_cast<V*>(y), g, RW, lin_z_host[i], tw1,
                       tlo, thi);
    LDBP_HIP_CHECK(hipGetLastError());
  }
  return LDBP_OK;
}

int ssm_run(int dtype, const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
            const std::vector<SsmPw>& pw, const void* noise, void* ws, hipStream_t s) {
  const int32_t M = static_cast<int32_t>(lin_z.size());
  // workspace: [lin_z (M doubles)] [ops (M+1 PwOp)] [tables]
  char* base = static_cast<char*>(ws);
  double* zdev = reinterpret_cast<double*>(base);
  const size_t zbytes = (static_cast<size_t>(M) * sizeof(double) + 255) & ~size_t(255);
  PwOp* odev = reinterpret_cast<PwOp*>(base + zbytes);
  const size_t obytes = ((static_cast<size_t>(M) + 1) * sizeof(PwOp) + 255) & ~size_t(255);
  void* tables = base + zbytes + obytes;
  std::vector<PwOp> ops(M + 1);
  for (int i = 0; i <= M; ++i) ops[i] = PwOp{pw[i].ka, pw[i].g, pw[i].sigma, pw[i].kb, pw[i].slot, 0};
  if (M > 0) LDBP_HIP_CHECK(hipMemcpyAsync(zdev, lin_z.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  LDBP_HIP_CHECK(hipMemcpyAsync(odev, ops.data(), (M + 1) * sizeof(PwOp), hipMemcpyHostToDevice, s));
  // the host vectors are copied before hipMemcpyAsync returns for pageable memory; synchronise the
  // stream anyway so the host buffers may be released safely
  LDBP_HIP_CHECK(hipStreamSynchronize(s));
  if (dtype == LDBP_C64) return run_t<float>(g, x, y, zdev, odev, M, lin_z, noise, tables, s);
  return run_t<double>(g, x, y, zdev, odev, M, lin_z, noise, tables, s);
}

size_t ssm_workspace_bytes(int dtype, const SsmGeom& g, int32_t M) {
  const size_t zbytes = (static_cast<size_t>(M) * sizeof(double) + 255) & ~size_t(255);
  const size_t obytes = ((static_cast<size_t>(M) + 1) * sizeof(PwOp) + 255) & ~size_t(255);
  return zbytes + obytes + ssm_table_elems(g) * elem_size(dtype);
}

size_t ssm_lds_bytes(int dtype, const SsmGeom& g) {
  if (g.resident) return 2 * static_cast<size_t>(g.n) * g.npol * elem_size(dtype);
  const int E = tile_elems(dtype, g);
  const int C = std::max(1, std::min<int>(g.N1, E / (g.N2 * g.npol)));
  const int RW = std::max(1, std::min<int>(g.N2, E / (g.N1 * g.npol)));
  return 2 * std::max(static_cast<size_t>(g.N2) * C, static_cast<size_t>(g.N1) * RW) * g.npol * elem_size(dtype);
}

}  // namespace ldbp
