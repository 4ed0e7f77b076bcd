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
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.h"
#include "fft.h"
#include "bufio.h"
#include "team_fft.h"
#include "ssm_kernels.h"
#include "ssm_ops.h"

namespace ldbp {

constexpr int kSsmThreads = 256;

// amp * exp(2 pi i rev) for |rev| <= 1/2
template <typename R>
__device__ __forceinline__ cx_t<R> rev_phasor(double rev, R amp) {
  R s, c;
  if constexpr (sizeof(R) == 4) {
    Rot32::sincos_rev(static_cast<float>(rev), s, c);
  } else {
    sincospi(2.0 * rev, &s, &c);
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

// Up to six such tables written back to back by one launch.
struct TwSegs {
  int64_t count[6], mult[6], len[6];
  int32_t nseg;
};

template <typename R>
__global__ void twiddle_tables(cx_t<R>* __restrict__ tab, TwSegs sg) {
  int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  int64_t off = 0;
  for (int i = 0; i < sg.nseg; ++i) {
    if (k < sg.count[i]) {
      const int64_t e = (k * sg.mult[i]) % sg.len[i];
      double s, c;
      sincospi(-2.0 * static_cast<double>(e) / static_cast<double>(sg.len[i]), &s, &c);
      tab[off + k] = cx_t<R>{static_cast<R>(c), static_cast<R>(s)};
      return;
    }
    k -= sg.count[i];
    off += sg.count[i];
  }
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
    // (the polarisation count is a literal in each branch, so the sample stays in registers)
    if (np == 1) {
      for (int t = threadIdx.x; t < n; t += kSsmThreads) {
        V v[1] = {A[t]};
        apply_pw<R>(v, 1, op, nz ? nz + t : nullptr);
        A[t] = v[0];
      }
    } else {
      for (int t = threadIdx.x; t < n; t += kSsmThreads) {
        V v[2] = {A[2 * t], A[2 * t + 1]};
        apply_pw<R>(v, 2, op, nz ? nz + static_cast<int64_t>(t) * 2 : nullptr);
        A[2 * t] = v[0];
        A[2 * t + 1] = v[1];
      }
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
//
// Both passes keep a waveform tile in registers: a team of N/16 lanes holds one length-N sequence
// (a column for the column pass, a row for the row pass), 16 values per lane, element e in lane
// e mod (N/16), register e / (N/16); see team_fft.h.  A workgroup is 256 lanes.

constexpr int kSsmPassThreads = 256;
// waves per SIMD the passes are compiled for: in FP32 4 (<= 128 VGPRs) up to length 256 and 3 beyond,
// in FP64 2
template <typename R, int LOG2L>
constexpr int kPassMinWaves = sizeof(R) == 4 ? (LOG2L <= 8 ? 4 : 3) : 2;

// Kerr phase of one lane's value; with two polarisations the partner lane (lane ^ 1) holds the other
// polarisation of the same time sample.
template <typename R>
__device__ __forceinline__ cx_t<R> kerr_lane(cx_t<R> v, int npol, double k) {
  R p = v.x * v.x + v.y * v.y;
  if (npol == 2) p += __shfl_xor(p, 1);
  R s, c;
  phase_sincos(static_cast<R>(k) * phase_coef_scale<R>(), p, s, c);
  return cx_t<R>{v.x * c - v.y * s, v.x * s + v.y * c};
}

template <typename R>
__device__ __forceinline__ cx_t<R> twiddle_n(int64_t e, int lo_log, const cx_t<R>* __restrict__ tlo,
                                             const cx_t<R>* __restrict__ thi) {
  const cx_t<R> a = tlo[e & ((int64_t(1) << lo_log) - 1)];
  const cx_t<R> b = thi[e >> lo_log];
  return cmul_t(a, b);
}

// The four-step twiddles W_n^(t1 (t + T m)), m = 0..15, of one column lane, as a = W_n^(t1 t) times
// powers of b = W_n^(t1 T): b, b^2, b^4, b^8 come from the table, and the twiddle of m is the one of
// m minus its lowest set bit times that power, so each is a product of at most five table values.
template <typename R>
struct ColTwiddles {
  cx_t<R> a, b1, b2, b4, b8;
};

template <typename R>
__device__ __forceinline__ ColTwiddles<R> col_twiddles(int64_t t1, int t, int T, const SsmGeom& g,
                                                       const cx_t<R>* __restrict__ tlo,
                                                       const cx_t<R>* __restrict__ thi) {
  const int64_t mask = g.n - 1;
  const int64_t e = (t1 * T) & mask;
  return ColTwiddles<R>{twiddle_n<R>(t1 * t, g.lo_log, tlo, thi), twiddle_n<R>(e, g.lo_log, tlo, thi),
                        twiddle_n<R>((2 * e) & mask, g.lo_log, tlo, thi),
                        twiddle_n<R>((4 * e) & mask, g.lo_log, tlo, thi),
                        twiddle_n<R>((8 * e) & mask, g.lo_log, tlo, thi)};
}

template <typename R, bool CONJ>
__device__ __forceinline__ void apply_col_twiddles(cx_t<R> (&v)[kTeamLanes], const ColTwiddles<R>& c) {
  using V = cx_t<R>;
  V p[kTeamLanes];
  p[0] = c.a;
#pragma unroll
  for (int m = 1; m < kTeamLanes; ++m) {
    const int lb = m & -m;
    p[m] = cmul_t(p[m - lb], lb == 1 ? c.b1 : lb == 2 ? c.b2 : lb == 4 ? c.b4 : c.b8);
  }
#pragma unroll
  for (int m = 0; m < kTeamLanes; ++m) {
    V w = p[m];
    if (CONJ) w.y = -w.y;
    v[m] = cmul_t(v[m], w);
  }
}

template <typename R>
__device__ __forceinline__ void stage_table(cx_t<R>* dst, const cx_t<R>* __restrict__ src, int count) {
  for (int k = threadIdx.x; k < count; k += kSsmPassThreads) dst[k] = src[k];
}

template <int LOG2N2>
__host__ __device__ constexpr int col_teams() {
  return kSsmPassThreads / (1 << (LOG2N2 - 4));
}
template <int LOG2N2>
__host__ __device__ constexpr int col_pad() {
  return col_teams<LOG2N2>() < 32 ? col_teams<LOG2N2>() : 0;
}
template <int LOG2N2>
__host__ __device__ constexpr int col_xch_elems() {
  return (1 << LOG2N2) * col_teams<LOG2N2>() + ((1 << LOG2N2) >> 4) * col_pad<LOG2N2>();
}

// Column pass.  A workgroup takes G = 256 / T2 consecutive (column, polarisation) sequences of one
// waveform (T2 = N2/16 lanes each, lanes of a team G apart so that a load instruction reads G
// consecutive elements of a row).  One program step: the conjugate four-step twiddle W_n^(-t1 f2) and
// the inverse column FFT over f2 of the previous step (do_ifft), the pointwise operation P_i in the
// time domain, the forward column FFT over t2 and the twiddle W_n^(t1 f2) (do_fft).  The twiddles of
// both directions belong to this pass, so the row pass needs none.
template <typename R, int LOG2N2>
__global__ __launch_bounds__(kSsmPassThreads, (kPassMinWaves<R, LOG2N2>)) void ssm_col_kernel(
    const cx_t<R>* src, cx_t<R>* dst, SsmGeom g, PwOp op, int32_t do_ifft, int32_t do_fft,
    const cx_t<R>* __restrict__ noise, const cx_t<R>* __restrict__ tw2g, const cx_t<R>* __restrict__ tlo,
    const cx_t<R>* __restrict__ thi) {
  using V = cx_t<R>;
  constexpr int T = 1 << (LOG2N2 - 4);
  constexpr int G = col_teams<LOG2N2>();
  extern __shared__ __align__(16) unsigned char smem[];
  V* xb = reinterpret_cast<V*>(smem);
  V* tw = xb + col_xch_elems<LOG2N2>();
  const int np = g.npol;
  const int rowlen = g.N1 * np;  // elements in one row t2 (or f2)
  const int nblk = rowlen / G;
  const int cb = static_cast<int>(blockIdx.x % static_cast<uint32_t>(nblk));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(nblk);
  const int w = threadIdx.x % G;  // team: (column, polarisation) within the tile
  const int t = threadIdx.x / G;  // lane within the team
  // the tile: G consecutive elements of each of the N2 rows, from element `reg` of the batch
  const int64_t reg = wave * g.n * np + static_cast<int64_t>(cb) * G;
  const uint32_t span = static_cast<uint32_t>((static_cast<int64_t>(g.N2 - 1) * rowlen + G) * sizeof(V));
  const uint32_t voff = static_cast<uint32_t>((w + static_cast<int64_t>(t) * rowlen) * sizeof(V));
  const uint32_t mstep = static_cast<uint32_t>(static_cast<int64_t>(T) * rowlen * sizeof(V));
  const int64_t t1 = (static_cast<int64_t>(cb) * G + w) / np;
  const XchInterleaved<V> xc{xb, G, col_pad<LOG2N2>(), w};
  stage_table<R>(tw, tw2g, team_tw_entries(LOG2N2));
  V v[kTeamLanes];
  {
    const auto rs = make_rsrc(src + reg, span);
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) v[m] = buf_load<R>(rs, voff, m * mstep);
  }
  __syncthreads();
  if (do_ifft) {
    apply_col_twiddles<R, true>(v, col_twiddles<R>(t1, t, T, g, tlo, thi));
    team_fft<R, -1, LOG2N2>(v, t, xc, tw);
  }
  if (op.ka != 0.0) {
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) v[m] = kerr_lane<R>(v[m], np, op.ka);
  }
  if (op.g != 1.0) {
    const R gg = static_cast<R>(op.g);
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) v[m] = V{v[m].x * gg, v[m].y * gg};
  }
  if (op.slot >= 0 && noise) {
    const auto rn = make_rsrc(noise + static_cast<int64_t>(op.slot) * g.nwave * g.n * np + reg, span);
    const R sg = static_cast<R>(op.sigma);
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) {
      const V e = buf_load<R>(rn, voff, m * mstep);
      v[m] = V{v[m].x + sg * e.x, v[m].y + sg * e.y};
    }
  }
  if (op.kb != 0.0) {
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) v[m] = kerr_lane<R>(v[m], np, op.kb);
  }
  if (do_fft) {
    team_fft<R, 1, LOG2N2>(v, t, xc, tw);
    apply_col_twiddles<R, false>(v, col_twiddles<R>(t1, t, T, g, tlo, thi));
  }
  const auto rd = make_rsrc(dst + reg, span);
#pragma unroll
  for (int m = 0; m < kTeamLanes; ++m) buf_store<R>(v[m], rd, voff, m * mstep);
}

template <int LOG2N1>
__host__ __device__ constexpr int row_teams() {
  return kSsmPassThreads / (1 << (LOG2N1 - 4));
}
template <int LOG2N1>
__host__ __device__ constexpr int row_stride() {
  return (1 << LOG2N1) + 16;
}

// Row pass, in place.  A team of T1 = N1/16 consecutive lanes takes one (row f2, polarisation)
// sequence: forward FFT over t1 -> f1 (bin k = f2 + N2 f1), the step response times 1/n and the
// inverse FFT back to t1.
template <typename R, int LOG2N1>
__global__ __launch_bounds__(kSsmPassThreads, (kPassMinWaves<R, LOG2N1>)) void ssm_row_kernel(cx_t<R>* __restrict__ data,
                                                                                    SsmGeom g, double z,
                                                                                    const cx_t<R>* __restrict__ tw1g) {
  using V = cx_t<R>;
  constexpr int T = 1 << (LOG2N1 - 4);
  constexpr int GR = row_teams<LOG2N1>();
  extern __shared__ __align__(16) unsigned char smem[];
  V* xb = reinterpret_cast<V*>(smem);
  V* tw = xb + GR * row_stride<LOG2N1>();
  const int np = g.npol;
  const int t = threadIdx.x % T;
  const int gi = threadIdx.x / T;  // team (row, polarisation) in the workgroup, polarisation fastest
  const int rows = GR / np;        // rows per workgroup; they lie in one waveform
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows;  // global row wave * N2 + f2
  const int64_t f2 = row0 % g.N2 + gi / np;
  const int rowlen = g.N1 * np;
  const auto rs = make_rsrc(data + row0 * rowlen, static_cast<uint32_t>(static_cast<int64_t>(rows) * rowlen * sizeof(V)));
  const uint32_t voff = static_cast<uint32_t>(((gi / np) * rowlen + t * np + gi % np) * sizeof(V));
  const uint32_t mstep = static_cast<uint32_t>(T * np * sizeof(V));
  const XchTeamMajor<V> xc{xb, row_stride<LOG2N1>(), gi};
  stage_table<R>(tw, tw1g, team_tw_entries(LOG2N1));
  V v[kTeamLanes];
#pragma unroll
  for (int m = 0; m < kTeamLanes; ++m) v[m] = buf_load<R>(rs, voff, m * mstep);
  __syncthreads();
  team_fft<R, 1, LOG2N1>(v, t, xc, tw);
  // step response of bin k = f2 + N2 (t + T m): its signed index is k0 + D j with k0 = f2 + N2 t < D = n/16
  // and j = m (m < 8) or m - 16, so the phase zrev (k0 + D j)^2 revolutions is A + j B + j^2 C with
  // the three per-lane terms reduced modulo one in FP64
  const double zrev = z * g.beta2 * M_PI * g.fs * g.fs / (static_cast<double>(g.n) * g.n);
  const R amp = static_cast<R>(exp(-0.5 * z * g.alpha) / static_cast<double>(g.n));
  {
    const double k0 = static_cast<double>(f2 + static_cast<int64_t>(g.N2) * t);
    const double D = static_cast<double>(g.n / 16);
    double A = zrev * k0 * k0, B = 2.0 * zrev * k0 * D, C = zrev * D * D;
    A -= rint(A);
    B -= rint(B);
    C -= rint(C);
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) {
      const double j = m < kTeamLanes / 2 ? m : m - kTeamLanes;
      double rev = A + j * B + (j * j) * C;
      rev -= rint(rev);
      v[m] = cmul_t(v[m], rev_phasor<R>(rev, amp));
    }
  }
  team_fft<R, -1, LOG2N1>(v, t, xc, tw);
#pragma unroll
  for (int m = 0; m < kTeamLanes; ++m) buf_store<R>(v[m], rs, voff, m * mstep);
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
  } else if ((n & (n - 1)) != 0) {
    // not a power of two: mixed-radix passes, their own split (ssm_var.hip)
    g.resident = 0;
    g.mixed = 1;
    VarWave w;
    if (var_geometry(dtype, npol, n, w, nullptr) == LDBP_OK) {
      g.N1 = w.N1;
      g.N2 = w.N2;
    }
  } else {
    // N2 = 256 columns of length 256 up to n = 2^16; beyond, rows grow to 4096 / npol elements
    // (the row pass holds one row of every polarisation in a 256-lane workgroup) and columns take the rest
    g.resident = 0;
    int64_t N2 = n >= (int64_t(1) << 16) ? 256 : n / 256;
    if ((n / N2) * npol > 4096) N2 = n * npol / 4096;
    g.N2 = static_cast<int32_t>(N2);
    g.N1 = static_cast<int32_t>(n / N2);
  }
  g.lo_log = (ilog2(n) + 1) / 2;
  return g;
}

size_t ssm_table_elems(const SsmGeom& g) {
  if (g.resident) return static_cast<size_t>(g.n);
  if (g.mixed) return 0;
  return static_cast<size_t>(team_tw_entries(ilog2(g.N1))) + team_tw_entries(ilog2(g.N2)) +
         (int64_t(1) << g.lo_log) + (g.n >> g.lo_log);
}

static size_t elem_size(int dtype) { return cx_size(dtype); }

template <typename R, int LOG2N2>
static size_t col_lds() {
  return (static_cast<size_t>(col_xch_elems<LOG2N2>()) + team_tw_entries(LOG2N2)) * sizeof(cx_t<R>);
}
template <typename R, int LOG2N1>
static size_t row_lds() {
  return (static_cast<size_t>(row_teams<LOG2N1>()) * row_stride<LOG2N1>() + team_tw_entries(LOG2N1)) *
         sizeof(cx_t<R>);
}

// Kernels and LDS bytes of the four-step passes for one (N2, N1) split.
template <typename R>
struct FourStep {
  using V = cx_t<R>;
  using ColFn = void (*)(const V*, V*, SsmGeom, PwOp, int32_t, int32_t, const V*, const V*, const V*, const V*);
  using RowFn = void (*)(V*, SsmGeom, double, const V*);
  ColFn col = nullptr;
  RowFn row = nullptr;
  size_t col_bytes = 0, row_bytes = 0;
};

template <typename R, int L2>
static void pick_col(FourStep<R>& f) {
  f.col = ssm_col_kernel<R, L2>;
  f.col_bytes = col_lds<R, L2>();
}
template <typename R, int L1>
static void pick_row(FourStep<R>& f) {
  f.row = ssm_row_kernel<R, L1>;
  f.row_bytes = row_lds<R, L1>();
}

template <typename R>
static bool four_step(const SsmGeom& g, FourStep<R>& f) {
  switch (ilog2(g.N2)) {
    case 4: pick_col<R, 4>(f); break;
    case 5: pick_col<R, 5>(f); break;
    case 6: pick_col<R, 6>(f); break;
    case 7: pick_col<R, 7>(f); break;
    case 8: pick_col<R, 8>(f); break;
    case 9: pick_col<R, 9>(f); break;
    case 10: pick_col<R, 10>(f); break;
    case 11: pick_col<R, 11>(f); break;
    case 12: pick_col<R, 12>(f); break;
    default: return false;
  }
  switch (ilog2(g.N1)) {
    case 8: pick_row<R, 8>(f); break;
    case 9: pick_row<R, 9>(f); break;
    case 10: pick_row<R, 10>(f); break;
    case 11: pick_row<R, 11>(f); break;
    case 12: pick_row<R, 12>(f); break;
    default: return false;
  }
  // a column tile is G = 256 / (N2/16) sequences of one row and must hold both polarisations of its
  // columns (the Kerr phase pairs lane w with lane w ^ 1); a row workgroup holds 4096 / N1 sequences
  const int G = kSsmPassThreads / (g.N2 / 16);
  return G % g.npol == 0 && (static_cast<int64_t>(g.N1) * g.npol) % G == 0 &&
         static_cast<int64_t>(g.N1) * g.npol <= 4096 && (g.n * g.npol) % 4096 == 0;
}

template <typename R>
static int gen_tables(cx_t<R>* tab, const TwSegs& sg, hipStream_t s) {
  int64_t total = 0;
  for (int i = 0; i < sg.nseg; ++i) total += sg.count[i];
  hipLaunchKernelGGL(twiddle_tables<R>, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, s, tab, sg);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

// Resident path: the whole program runs in one launch, which reads the step list from the workspace.
template <typename R>
static int run_resident(const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
                        const std::vector<PwOp>& ops, const void* noise, void* ws, hipStream_t s) {
  using V = cx_t<R>;
  const int32_t M = static_cast<int32_t>(lin_z.size());
  char* base = static_cast<char*>(ws);
  double* zdev = reinterpret_cast<double*>(base);
  const size_t zbytes = (static_cast<size_t>(M) * sizeof(double) + 255) & ~size_t(255);
  PwOp* odev = reinterpret_cast<PwOp*>(base + zbytes);
  const size_t obytes = ((static_cast<size_t>(M) + 1) * sizeof(PwOp) + 255) & ~size_t(255);
  V* tab = reinterpret_cast<V*>(base + zbytes + obytes);
  // The program goes to the device from a heap copy that a host function queued behind the copy frees,
  // so the call returns without waiting for the stream (the caller's vectors are released on return).
  {
    auto* prog = new std::vector<char>(zbytes + obytes);
    if (M > 0) std::memcpy(prog->data(), lin_z.data(), M * sizeof(double));
    std::memcpy(prog->data() + zbytes, ops.data(), (M + 1) * sizeof(PwOp));
    hipError_t e = hipMemcpyAsync(base, prog->data(), prog->size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipLaunchHostFunc(s, [](void* p) { delete static_cast<std::vector<char>*>(p); }, prog);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      delete prog;
      return fail(LDBP_EHIP, "copying the split-step program: %s", hipGetErrorString(e));
    }
  }
  TwSegs sg{};
  sg.nseg = 1;
  sg.count[0] = g.n;
  sg.mult[0] = 1;
  sg.len[0] = g.n;
  int st = gen_tables<R>(tab, sg, s);
  if (st) return st;
  const size_t lds = 2 * static_cast<size_t>(g.n) * g.npol * sizeof(V);
  auto kern = ssm_resident_kernel<R>;
  if (lds > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(g.nwave)), dim3(kSsmThreads), lds, s, static_cast<const V*>(x),
                     static_cast<V*>(y), g, zdev, odev, M, static_cast<const V*>(noise), tab);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

// Four-step path: one column and one row launch per step; the pointwise operation and the step length
// travel as kernel arguments, so nothing but the twiddle tables is staged in the workspace.
template <typename R>
static int run_four_step(const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
                         const std::vector<PwOp>& ops, const void* noise, void* ws, hipStream_t s) {
  using V = cx_t<R>;
  const int32_t M = static_cast<int32_t>(lin_z.size());
  FourStep<R> fs;
  if (!four_step<R>(g, fs)) return fail(LDBP_EUNSUPPORTED, "no four-step split for n = %lld", (long long)g.n);
  const int l1 = ilog2(g.N1), l2 = ilog2(g.N2);
  V* tw1 = static_cast<V*>(ws);
  V* tw2 = tw1 + team_tw_entries(l1);
  V* tlo = tw2 + team_tw_entries(l2);
  V* thi = tlo + (int64_t(1) << g.lo_log);
  // team tables for N1 and N2 (a two-level one is W_L^k for k < 2^LB followed by W_L^(k 2^LB)), then
  // W_n in two levels, written back to back by one launch
  TwSegs sg{};
  auto add = [&](int64_t count, int64_t mult, int64_t len) {
    sg.count[sg.nseg] = count;
    sg.mult[sg.nseg] = mult;
    sg.len[sg.nseg] = len;
    ++sg.nseg;
  };
  for (const int lg : {l1, l2}) {
    const int lb = team_tw_lb(lg);
    add(int64_t(1) << lb, 1, int64_t(1) << lg);
    if (lb < lg) add(int64_t(1) << (lg - lb), int64_t(1) << lb, int64_t(1) << lg);
  }
  add(int64_t(1) << g.lo_log, 1, g.n);
  add(g.n >> g.lo_log, int64_t(1) << g.lo_log, g.n);
  const int st = gen_tables<R>(tw1, sg, s);
  if (st) return st;
  if (fs.col_bytes > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fs.col),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(fs.col_bytes)));
  if (fs.row_bytes > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fs.row),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(fs.row_bytes)));
  const int G = kSsmPassThreads / (g.N2 / 16);
  const uint32_t gc = static_cast<uint32_t>((static_cast<int64_t>(g.N1) * g.npol / G) * g.nwave);
  const uint32_t gr = static_cast<uint32_t>(g.n * g.npol * g.nwave / 4096);
  const V* nz = static_cast<const V*>(noise);
  for (int i = 0; i <= M; ++i) {
    const V* src = (i == 0) ? static_cast<const V*>(x) : static_cast<const V*>(y);
    hipLaunchKernelGGL(fs.col, dim3(gc), dim3(kSsmPassThreads), fs.col_bytes, s, src, static_cast<V*>(y), g, ops[i],
                       i > 0 ? 1 : 0, i < M ? 1 : 0, nz, tw2, tlo, thi);
    LDBP_HIP_CHECK(hipGetLastError());
    if (i == M) break;
    hipLaunchKernelGGL(fs.row, dim3(gr), dim3(kSsmPassThreads), fs.row_bytes, s, static_cast<V*>(y), g, lin_z[i],
                       tw1);
    LDBP_HIP_CHECK(hipGetLastError());
  }
  return LDBP_OK;
}

int ssm_run(int dtype, const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
            const std::vector<SsmPw>& pw, const void* noise, void* ws, hipStream_t s) {
  const int32_t M = static_cast<int32_t>(lin_z.size());
  std::vector<PwOp> ops(M + 1);
  for (int i = 0; i <= M; ++i) ops[i] = PwOp{pw[i].ka, pw[i].g, pw[i].sigma, pw[i].kb, pw[i].slot, 0};
  if (g.resident) {
    if (dtype == LDBP_C64) return run_resident<float>(g, x, y, lin_z, ops, noise, ws, s);
    return run_resident<double>(g, x, y, lin_z, ops, noise, ws, s);
  }
  if (g.mixed) return ssm_run_var(dtype, g, x, y, lin_z, pw, noise, ws, s);
  if (dtype == LDBP_C64) return run_four_step<float>(g, x, y, lin_z, ops, noise, ws, s);
  return run_four_step<double>(g, x, y, lin_z, ops, noise, ws, s);
}

size_t ssm_workspace_bytes(int dtype, const SsmGeom& g, int32_t M) {
  if (g.mixed) return ssm_var_workspace_bytes(dtype, g.npol, g.n);
  if (!g.resident) return ssm_table_elems(g) * elem_size(dtype);
  const size_t zbytes = (static_cast<size_t>(M) * sizeof(double) + 255) & ~size_t(255);
  const size_t obytes = ((static_cast<size_t>(M) + 1) * sizeof(PwOp) + 255) & ~size_t(255);
  return zbytes + obytes + ssm_table_elems(g) * elem_size(dtype);
}

size_t ssm_lds_bytes(int dtype, const SsmGeom& g) {
  if (g.resident) return 2 * static_cast<size_t>(g.n) * g.npol * elem_size(dtype);
  if (g.mixed) return ssm_var_lds_bytes(dtype, g.npol, g.n);
  if (dtype == LDBP_C64) {
    FourStep<float> f;
    if (!four_step<float>(g, f)) return ~size_t(0);
    return std::max(f.col_bytes, f.row_bytes);
  }
  FourStep<double> f;
  if (!four_step<double>(g, f)) return ~size_t(0);
  return std::max(f.col_bytes, f.row_bytes);
}

}  // namespace ldbp
