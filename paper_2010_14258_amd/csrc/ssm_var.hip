// Split-step engine for lengths whose prime factors are 2, 3 and 5 (Sec. III-A: the DFT grid of the
// time-discretised NLSE has any length), and for batches whose waveforms differ in length and in
// step program (the uneven serving batch of FFT-based DBP).
//
// Same four-step structure as the power-of-two passes of ssm.hip (position t = t1 + N1 t2,
// frequency k = f2 + N2 f1, memory holding the column-transformed and twiddled values at t1 + N1 f2
// between passes), but the transforms are mixed-radix Stockham FFTs in LDS (fft.h) over tiles:
//   column pass  a tile of C consecutive columns t1 (all polarisations), N2 x C x npol values:
//                conjugate twiddle W_n^(-t1 f2) and inverse FFT over f2 (from the second program
//                step on), the pointwise operation P_i in the time domain, forward FFT over t2 and
//                twiddle W_n^(t1 f2) (up to the last linear step);
//   row pass     a tile of RW consecutive rows f2, N1 x RW x npol values: forward FFT over t1, the
//                step response exp(z (j beta2 w_k^2/2 - alpha/2)) / n at bin k = f2 + N2 f1, inverse
//                FFT, in place.
// A launch covers work items (waveform, tile); the waveforms of a batch plan are sorted by their
// number of linear steps, so the launch of program step i covers a prefix of the item lists (the
// waveforms that still have step i).  A uniform batch (one length and program) needs no device
// tables: its items follow from the block index, its operation and step length are kernel
// arguments.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "fft.h"
#include "ssm_kernels.h"
#include "ssm_ops.h"

namespace ldbp {

constexpr int kVarThreads = 256;
// complex values per LDS buffer of a tile (two buffers per tile, plus the twiddle table of the pass's
// transform length): the smallest of these that admits a split n = N1 N2 with N1, N2 <= E / npol, so
// that two or three workgroups fit on a compute unit
constexpr int kVarTileElems[] = {2048, 4096};
constexpr size_t kVarMaxLds = 160 * 1024;

struct VarArgs {
  const VarWave* waves;  // per-waveform geometry, NULL for a uniform batch (then `uni`)
  const VarItem* items;  // work items of the launch, NULL for a uniform batch (items from the block index)
  const double* z;       // per-waveform programs: step lengths ...
  const PwOp* ops;       // ... and pointwise operations (NULL for a uniform batch: `op`, `zstep`)
  const void* noise;     // noise slots, slot s at noise + s * noise_slot (complex values)
  const void* tab;       // twiddle tables (complex of the dtype)
  int64_t noise_slot;
  VarWave uni;
  PwOp op;
  double zstep;
  double fs, alpha, beta2;
  int32_t npol;
  int32_t pad;
};

template <typename R>
__device__ __forceinline__ cx_t<R> tw_n(const cx_t<R>* tab, const VarWave& w, int64_t e) {
  const cx_t<R> a = tab[w.tlo + (e & ((int64_t(1) << w.lo_log) - 1))];
  const cx_t<R> b = tab[w.thi + (e >> w.lo_log)];
  return cx_t<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename R>
__device__ __forceinline__ void var_item(const VarArgs& a, int tiles_field, VarWave& w, int& tile) {
  if (a.items) {
    const VarItem it = a.items[blockIdx.x];
    w = a.waves[it.wave];
    tile = it.tile;
  } else {
    w = a.uni;
    const int per = tiles_field == 0 ? w.ctiles : w.rtiles;
    const int wave = static_cast<int>(blockIdx.x / static_cast<uint32_t>(per));
    tile = static_cast<int>(blockIdx.x) - wave * per;
    w.off = static_cast<int64_t>(wave) * w.n * a.npol;
  }
}

// Column pass of program step `step` (see the file comment); src -> dst, same positions.
template <typename R>
__global__ __launch_bounds__(kVarThreads) void ssm_var_col(const cx_t<R>* src, cx_t<R>* dst, VarArgs a,
                                                           int32_t step) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  VarWave w;
  int tile;
  var_item<R>(a, 0, w, tile);
  const int np = a.npol, plog = np - 1;
  const int C = w.C, width = C * np, wlog = __builtin_ctz(static_cast<unsigned>(width));
  const int N1 = w.N1, N2 = w.N2, c0 = tile * C;
  const V* tab = static_cast<const V*>(a.tab);
  const PwOp op = a.ops ? a.ops[w.prog_op + step] : a.op;
  const bool do_ifft = step > 0, do_fft = step < w.M;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N2) * width;
  V* tw = B + static_cast<size_t>(N2) * width;   // W_N2^k, k < N2, staged from the table buffer
  const int tot = N2 * width;
  const int64_t base = w.off + static_cast<int64_t>(c0) * np;
  for (int k = threadIdx.x; k < N2; k += kVarThreads) tw[k] = tab[w.tw2 + k];
  for (int e = threadIdx.x; e < tot; e += kVarThreads) {
    const int t2 = e >> wlog, q = e & (width - 1);
    V v{0, 0};
    if (c0 + (q >> plog) < N1) {
      v = src[base + static_cast<int64_t>(t2) * N1 * np + q];
      if (do_ifft) {
        V t = tw_n<R>(tab, w, static_cast<int64_t>(c0 + (q >> plog)) * t2);
        v = V{v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y};   // times conj(W_n^(t1 f2))
      }
    }
    A[e] = v;
  }
  __syncthreads();
  V* cur = A;
  V* oth = B;
  if (do_ifft) {
    cur = lds_fft_plan<R, -1, kVarThreads, false, true>(A, B, N2, width, tw, w.plan2);
    oth = (cur == A) ? B : A;
  }
  // pointwise operation on every time sample (t2, t1) of the tile, all polarisations together
  const int clog = wlog - plog;
  const V* nz = nullptr;
  if (op.slot >= 0 && a.noise) nz = static_cast<const V*>(a.noise) + op.slot * a.noise_slot;
  // (the polarisation count is a literal in each branch, so the sample stays in registers)
  if (np == 1) {
    for (int e = threadIdx.x; e < N2 * C; e += kVarThreads) {
      const int t2 = e >> clog, cc = e & (C - 1);
      if (c0 + cc >= N1) continue;
      V v[1] = {cur[e]};
      apply_pw<R>(v, 1, op, nz ? nz + base + static_cast<int64_t>(t2) * N1 + cc : nullptr);
      cur[e] = v[0];
    }
  } else {
    for (int e = threadIdx.x; e < N2 * C; e += kVarThreads) {
      const int t2 = e >> clog, cc = e & (C - 1);
      if (c0 + cc >= N1) continue;
      V v[2] = {cur[2 * e], cur[2 * e + 1]};
      apply_pw<R>(v, 2, op, nz ? nz + base + (static_cast<int64_t>(t2) * N1 + cc) * 2 : nullptr);
      cur[2 * e] = v[0];
      cur[2 * e + 1] = v[1];
    }
  }
  __syncthreads();
  if (do_fft) cur = lds_fft_plan<R, 1, kVarThreads, false, true>(cur, oth, N2, width, tw, w.plan2);
  for (int e = threadIdx.x; e < tot; e += kVarThreads) {
    const int f2 = e >> wlog, q = e & (width - 1);
    if (c0 + (q >> plog) >= N1) continue;
    V v = cur[e];
    if (do_fft) v = cmul(v, tw_n<R>(tab, w, static_cast<int64_t>(c0 + (q >> plog)) * f2));
    dst[base + static_cast<int64_t>(f2) * N1 * np + q] = v;
  }
}

// Row pass of program step `step`, in place on `data`.
template <typename R>
__global__ __launch_bounds__(kVarThreads) void ssm_var_row(cx_t<R>* data, VarArgs a, int32_t step) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  VarWave w;
  int tile;
  var_item<R>(a, 1, w, tile);
  const int np = a.npol, plog = np - 1;
  const int RW = w.RW, width = RW * np, wlog = __builtin_ctz(static_cast<unsigned>(width));
  const int N1 = w.N1, N2 = w.N2, r0 = tile * RW;
  const int rows = min(RW, N2 - r0);
  const V* tab = static_cast<const V*>(a.tab);
  const double z = a.ops ? a.z[w.prog + step] : a.zstep;
  V* A = reinterpret_cast<V*>(smem);
  V* B = A + static_cast<size_t>(N1) * width;
  V* tw = B + static_cast<size_t>(N1) * width;   // W_N1^k, k < N1, staged from the table buffer
  for (int k = threadIdx.x; k < N1; k += kVarThreads) tw[k] = tab[w.tw1 + k];
  const int rowlen = N1 * np;
  V* row0 = data + w.off + static_cast<int64_t>(r0) * rowlen;
  for (int r = 0; r < RW; ++r) {
    for (int e = threadIdx.x; e < rowlen; e += kVarThreads)
      A[(e >> plog) * width + r * np + (e & plog)] = r < rows ? row0[static_cast<int64_t>(r) * rowlen + e] : V{0, 0};
  }
  __syncthreads();
  V* F = lds_fft_plan<R, 1, kVarThreads, false, true>(A, B, N1, width, tw, w.plan1);
  V* oth = (F == A) ? B : A;
  const double n = static_cast<double>(w.n);
  const double zrev = z * a.beta2 * M_PI * a.fs * a.fs / (n * n);
  const R amp = static_cast<R>(exp(-0.5 * z * a.alpha) / n);
  for (int e = threadIdx.x; e < N1 * width; e += kVarThreads) {
    const int f1 = e >> wlog, r = (e & (width - 1)) >> plog;
    const int64_t k = r0 + r + static_cast<int64_t>(N2) * f1;
    F[e] = cmul(F[e], lin_response<R>(k, w.n, zrev, amp));
  }
  __syncthreads();
  V* T = lds_fft_plan<R, -1, kVarThreads, false, true>(F, oth, N1, width, tw, w.plan1);
  for (int r = 0; r < rows; ++r) {
    for (int e = threadIdx.x; e < rowlen; e += kVarThreads)
      row0[static_cast<int64_t>(r) * rowlen + e] = T[(e >> plog) * width + r * np + (e & plog)];
  }
}

// ---------------------------------------------------------------- host side

bool smooth5(int64_t n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

static int ceil_log2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

static int floor_pow2(int64_t v) {
  int p = 1;
  while (2 * static_cast<int64_t>(p) <= v) p *= 2;
  return p;
}

int var_geometry(int dtype, int npol, int64_t n, VarWave& w, size_t* lds_bytes) {
  if (!smooth5(n) || n < 2)
    return fail(LDBP_EUNSUPPORTED, "n = %lld: FFT lengths must be 2^a 3^b 5^c >= 2", (long long)n);
  // rows of N1 <= E / npol values per polarisation; N2 the smallest divisor that allows it, so that
  // column tiles read long runs of every row
  int64_t N2 = 0, E = 0;
  for (int e : kVarTileElems) {
    const int64_t max1 = e / npol;
    for (int64_t d = 1; d <= max1 && d <= n; ++d)
      if (n % d == 0 && n / d <= max1) {
        N2 = d;
        break;
      }
    if (N2) {
      E = e;
      break;
    }
  }
  if (N2 == 0) return fail(LDBP_EUNSUPPORTED, "n = %lld has no split into rows and columns of <= %d", (long long)n,
                           kVarTileElems[1] / npol);
  const int64_t N1 = n / N2;
  w = VarWave{};
  w.n = n;
  w.N1 = static_cast<int32_t>(N1);
  w.N2 = static_cast<int32_t>(N2);
  w.C = std::min<int>(floor_pow2(std::max<int64_t>(1, E / (N2 * npol))), 1 << ceil_log2(N1));
  w.RW = std::min<int>(floor_pow2(std::max<int64_t>(1, E / (N1 * npol))), 1 << ceil_log2(N2));
  w.ctiles = static_cast<int32_t>((N1 + w.C - 1) / w.C);
  w.rtiles = static_cast<int32_t>((N2 + w.RW - 1) / w.RW);
  w.lo_log = (ceil_log2(n) + 1) / 2;
  w.plan1 = fft_radix_plan_composite(static_cast<int>(N1));
  w.plan2 = fft_radix_plan_composite(static_cast<int>(N2));
  const size_t lds = (2 * std::max<size_t>(static_cast<size_t>(N2) * w.C, static_cast<size_t>(N1) * w.RW) * npol +
                      static_cast<size_t>(std::max(N1, N2))) * cx_size(dtype);
  if (lds > kVarMaxLds)
    return fail(LDBP_EUNSUPPORTED, "n = %lld with npol = %d needs %zu bytes of LDS per tile (at most %zu)",
                (long long)n, npol, lds, kVarMaxLds);
  if (lds_bytes) *lds_bytes = lds;
  return LDBP_OK;
}

int64_t var_table_elems(const VarWave& w) {
  return static_cast<int64_t>(w.N1) + w.N2 + (int64_t(1) << w.lo_log) + ((w.n + (int64_t(1) << w.lo_log) - 1) >> w.lo_log);
}

// tab[k] = exp(-2 pi i (k mult mod len) / len) for k < count, in FP64, rounded once.
template <typename R>
__global__ void var_twiddles(cx_t<R>* __restrict__ tab, int64_t count, int64_t mult, int64_t len) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= count) return;
  double s, c;
  sincospi(-2.0 * static_cast<double>((k * mult) % len) / static_cast<double>(len), &s, &c);
  tab[k] = cx_t<R>{static_cast<R>(c), static_cast<R>(s)};
}

// Writes the four tables of w at tab + toff and records their offsets in w.
int var_tables(int dtype, VarWave& w, void* tab, int64_t toff, hipStream_t s) {
  const int64_t lo = int64_t(1) << w.lo_log;
  const int64_t segs[4][3] = {{w.N1, 1, w.N1}, {w.N2, 1, w.N2}, {lo, 1, w.n}, {(w.n + lo - 1) / lo, lo, w.n}};
  int64_t* offs[4] = {&w.tw1, &w.tw2, &w.tlo, &w.thi};
  for (int i = 0; i < 4; ++i) {
    *offs[i] = toff;
    const uint32_t blocks = static_cast<uint32_t>((segs[i][0] + 255) / 256);
    if (dtype == LDBP_C64)
      hipLaunchKernelGGL(var_twiddles<float>, dim3(blocks), dim3(256), 0, s, static_cast<cx_t<float>*>(tab) + toff,
                         segs[i][0], segs[i][1], segs[i][2]);
    else
      hipLaunchKernelGGL(var_twiddles<double>, dim3(blocks), dim3(256), 0, s,
                         static_cast<cx_t<double>*>(tab) + toff, segs[i][0], segs[i][1], segs[i][2]);
    LDBP_HIP_CHECK(hipGetLastError());
    toff += segs[i][0];
  }
  return LDBP_OK;
}

template <typename R>
static int var_launch(bool col, const void* src, void* dst, const VarArgs& a, int32_t step, uint32_t blocks,
                      size_t lds, hipStream_t s) {
  using V = cx_t<R>;
  if (blocks == 0) return LDBP_OK;
  if (col) {
    if (lds > 65536)
      LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(ssm_var_col<R>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(ssm_var_col<R>, dim3(blocks), dim3(kVarThreads), lds, s, static_cast<const V*>(src),
                       static_cast<V*>(dst), a, step);
  } else {
    if (lds > 65536)
      LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(ssm_var_row<R>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(ssm_var_row<R>, dim3(blocks), dim3(kVarThreads), lds, s, static_cast<V*>(dst), a, step);
  }
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

static int var_launch_any(int dtype, bool col, const void* src, void* dst, const VarArgs& a, int32_t step,
                          uint32_t blocks, size_t lds, hipStream_t s) {
  return dtype == LDBP_C64 ? var_launch<float>(col, src, dst, a, step, blocks, lds, s)
                           : var_launch<double>(col, src, dst, a, step, blocks, lds, s);
}

size_t ssm_var_workspace_bytes(int dtype, int npol, int64_t n) {
  VarWave w;
  if (var_geometry(dtype, npol, n, w, nullptr)) return 0;
  return static_cast<size_t>(var_table_elems(w)) * cx_size(dtype);
}

size_t ssm_var_lds_bytes(int dtype, int npol, int64_t n) {
  VarWave w;
  size_t lds = 0;
  if (var_geometry(dtype, npol, n, w, &lds)) return ~size_t(0);
  return lds;
}

// Uniform batch: nwave waveforms of n samples, one program; tables in ws; the operation and step
// length of each launch travel as kernel arguments (no host-to-device copy, no synchronisation).
int ssm_run_var(int dtype, const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
                const std::vector<SsmPw>& pw, const void* noise, void* ws, hipStream_t s) {
  VarWave w;
  size_t lds = 0;
  int st = var_geometry(dtype, g.npol, g.n, w, &lds);
  if (st) return st;
  w.M = static_cast<int32_t>(lin_z.size());
  st = var_tables(dtype, w, ws, 0, s);
  if (st) return st;
  VarArgs a{};
  a.uni = w;
  a.tab = ws;
  a.noise = noise;
  a.noise_slot = g.nwave * g.n * g.npol;
  a.fs = g.fs;
  a.alpha = g.alpha;
  a.beta2 = g.beta2;
  a.npol = g.npol;
  const uint32_t gc = static_cast<uint32_t>(w.ctiles * g.nwave);
  const uint32_t gr = static_cast<uint32_t>(w.rtiles * g.nwave);
  for (int i = 0; i <= w.M; ++i) {
    a.op = PwOp{pw[i].ka, pw[i].g, pw[i].sigma, pw[i].kb, pw[i].slot, 0};
    st = var_launch_any(dtype, true, i == 0 ? x : y, y, a, i, gc, lds, s);
    if (st) return st;
    if (i == w.M) break;
    a.zstep = lin_z[i];
    st = var_launch_any(dtype, false, y, y, a, i, gr, lds, s);
    if (st) return st;
  }
  return LDBP_OK;
}

// ---------------------------------------------------------------- batch plans (uneven waveforms)

struct SsmBatchPlanImpl {
  int dtype = 0, npol = 1, dev = -1;
  int64_t nwave = 0, total = 0, sample_steps = 0, noise_slot = 0;
  int32_t max_M = 0, max_slots = 0;
  size_t lds = 0;
  std::vector<uint32_t> col_count, row_count;  // items of the launches of step i
  VarWave* d_waves = nullptr;
  VarItem* d_col = nullptr;
  VarItem* d_row = nullptr;
  double* d_z = nullptr;
  PwOp* d_ops = nullptr;
  void* d_tab = nullptr;
  double fs = 0, alpha = 0, beta2 = 0;
};

int ssm_batch_build(int dtype, int npol, int64_t nwave, const int64_t* len, const std::vector<std::vector<double>>& z,
                    const std::vector<std::vector<SsmPw>>& pw, double fs, double alpha, double beta2, void** out) {
  auto* P = new SsmBatchPlanImpl();
  P->dtype = dtype;
  P->npol = npol;
  P->nwave = nwave;
  P->fs = fs;
  P->alpha = alpha;
  P->beta2 = beta2;
  std::vector<VarWave> waves(nwave);
  std::vector<double> zall;
  std::vector<PwOp> ops;
  int64_t tabn = 0;
  for (int64_t b = 0; b < nwave; ++b) {
    VarWave& w = waves[b];
    size_t lds = 0;
    int st = var_geometry(dtype, npol, len[b], w, &lds);
    if (st) {
      delete P;
      return st;
    }
    P->lds = std::max(P->lds, lds);
    w.off = P->total * npol;
    P->total += len[b];
    w.M = static_cast<int32_t>(z[b].size());
    w.prog = static_cast<int32_t>(zall.size());
    w.prog_op = static_cast<int32_t>(ops.size());
    zall.insert(zall.end(), z[b].begin(), z[b].end());
    for (const auto& p : pw[b]) {
      ops.push_back(PwOp{p.ka, p.g, p.sigma, p.kb, p.slot, 0});
      P->max_slots = std::max(P->max_slots, p.slot + 1);
    }
    P->max_M = std::max(P->max_M, w.M);
    P->sample_steps += len[b] * w.M;
    w.tw1 = tabn;  // provisional: offsets fixed by var_tables below
    tabn += var_table_elems(w);
  }
  P->noise_slot = P->total * npol;
  // items: waveforms by decreasing number of steps (stable), wave-major
  std::vector<int64_t> order(nwave);
  for (int64_t b = 0; b < nwave; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return waves[a].M > waves[b].M; });
  std::vector<VarItem> col, row;
  P->col_count.assign(P->max_M + 1, 0);
  P->row_count.assign(P->max_M + 1, 0);
  for (int64_t b : order) {
    const VarWave& w = waves[b];
    for (int t = 0; t < w.ctiles; ++t) col.push_back(VarItem{static_cast<int32_t>(b), t});
    for (int t = 0; t < w.rtiles; ++t) row.push_back(VarItem{static_cast<int32_t>(b), t});
    for (int i = 0; i <= w.M; ++i) P->col_count[i] += w.ctiles;
    for (int i = 0; i < w.M; ++i) P->row_count[i] += w.rtiles;
  }
  auto fail_free = [&](int st) {
    hipFree(P->d_waves);
    hipFree(P->d_col);
    hipFree(P->d_row);
    hipFree(P->d_z);
    hipFree(P->d_ops);
    hipFree(P->d_tab);
    delete P;
    return st;
  };
  if (hipGetDevice(&P->dev) != hipSuccess) return fail_free(fail(LDBP_EHIP, "hipGetDevice failed"));
  // twiddle tables, generated on the device at their offsets
  if (hipMalloc(&P->d_tab, static_cast<size_t>(tabn) * cx_size(dtype)) != hipSuccess)
    return fail_free(fail(LDBP_EHIP, "hipMalloc of %lld twiddles failed", (long long)tabn));
  int64_t toff = 0;
  for (auto& w : waves) {
    const int64_t te = var_table_elems(w);
    const int st = var_tables(dtype, w, P->d_tab, toff, nullptr);
    if (st) return fail_free(st);
    toff += te;
  }
  auto upload = [&](void** dst, const void* src, size_t bytes) -> int {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return fail(LDBP_EHIP, "hipMalloc failed");
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      return fail(LDBP_EHIP, "hipMemcpy failed");
    return LDBP_OK;
  };
  int st = upload(reinterpret_cast<void**>(&P->d_waves), waves.data(), waves.size() * sizeof(VarWave));
  if (!st) st = upload(reinterpret_cast<void**>(&P->d_col), col.data(), col.size() * sizeof(VarItem));
  if (!st) st = upload(reinterpret_cast<void**>(&P->d_row), row.data(), row.size() * sizeof(VarItem));
  if (!st) st = upload(reinterpret_cast<void**>(&P->d_z), zall.data(), zall.size() * sizeof(double));
  if (!st) st = upload(reinterpret_cast<void**>(&P->d_ops), ops.data(), ops.size() * sizeof(PwOp));
  if (!st && hipDeviceSynchronize() != hipSuccess) st = fail(LDBP_EHIP, "table generation failed");
  if (st) return fail_free(st);
  *out = P;
  return LDBP_OK;
}

void ssm_batch_free(void* plan) {
  auto* P = static_cast<SsmBatchPlanImpl*>(plan);
  if (!P) return;
  hipFree(P->d_waves);
  hipFree(P->d_col);
  hipFree(P->d_row);
  hipFree(P->d_z);
  hipFree(P->d_ops);
  hipFree(P->d_tab);
  delete P;
}

void ssm_batch_totals(const void* plan, int64_t* samples, int64_t* sample_steps, int32_t* max_steps,
                      int32_t* slots, int32_t* npol, int32_t* dtype, int32_t* dev) {
  const auto* P = static_cast<const SsmBatchPlanImpl*>(plan);
  if (samples) *samples = P->total;
  if (sample_steps) *sample_steps = P->sample_steps;
  if (max_steps) *max_steps = P->max_M;
  if (slots) *slots = P->max_slots;
  if (npol) *npol = P->npol;
  if (dtype) *dtype = P->dtype;
  if (dev) *dev = P->dev;
}

int ssm_batch_exec(const void* plan, const void* x, void* y, const void* noise, hipStream_t s) {
  const auto* P = static_cast<const SsmBatchPlanImpl*>(plan);
  VarArgs a{};
  a.waves = P->d_waves;
  a.z = P->d_z;
  a.ops = P->d_ops;
  a.noise = noise;
  a.noise_slot = P->noise_slot;
  a.tab = P->d_tab;
  a.fs = P->fs;
  a.alpha = P->alpha;
  a.beta2 = P->beta2;
  a.npol = P->npol;
  for (int i = 0; i <= P->max_M; ++i) {
    a.items = P->d_col;
    int st = var_launch_any(P->dtype, true, i == 0 ? x : y, y, a, i, P->col_count[i], P->lds, s);
    if (st) return st;
    if (i == P->max_M) break;
    a.items = P->d_row;
    st = var_launch_any(P->dtype, false, y, y, a, i, P->row_count[i], P->lds, s);
    if (st) return st;
  }
  return LDBP_OK;
}

}  // namespace ldbp
