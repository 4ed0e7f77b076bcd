// Batched LDBP inference over waveforms of uneven length, step count and filter length.
//
// Each waveform b (n_b samples, l_b steps, its own taps and Kerr coefficients) is processed with
// all of its steps fused in one pass: a workgroup loads a tile of L_b samples plus a halo of
// H_b = sum of K over the waveform's steps (circularly), runs the l_b FIR + Kerr steps in LDS and
// writes the L_b samples whose dependency cone it loaded (eq. model, Sec. III-B).  Work items
// (waveform, tile) are therefore independent: one launch covers the whole batch, items are
// ordered by decreasing cost so the hardware dispatcher balances the tail, and the launch can be
// captured once into a hipGraph and replayed.  A waveform whose halo does not leave a useful tile
// in the largest LDS work size runs its steps in groups, one further launch per group.
// Per-waveform and per-step tables (and the intermediate signal of such waveforms) live in device
// memory owned by the plan (allocated once when the plan is created).
#include <algorithm>
#include <numeric>
#include <vector>

#include "common.h"
#include "ldbp_fir.h"
#include "ldbp_kernels.h"

namespace ldbp {

// One pass over one waveform: all of its steps, or (a waveform whose halo leaves no tile in the LDS work
// size) one group of consecutive steps, reading the previous group's output.
struct BatchWave {
  int64_t off;       // first time sample of the waveform in the packed arrays
  int64_t toff;      // first time sample of the waveform in the plan's intermediate buffer
  int32_t n;         // samples
  int32_t nstep;     // steps of this pass
  int32_t step0;     // first entry in the step table
  int32_t halo;      // H_b: sum of K over the pass's steps
  int32_t tile_len;  // L_b
  int32_t wrap;      // 1 when H_b >= n_b
  int32_t src, dst;  // 0: x, 1: y, 2: the intermediate buffer
};

struct BatchStep {
  int32_t K;
  int32_t tapoff;  // into the packed taps of the whole batch
  int32_t cidx;    // into the packed Kerr coefficients
  int32_t pad;
};

struct BatchItem {
  int32_t wave;
  int32_t tile;
};

template <typename R, int NPOL, int RB, int THREADS>
__global__ __launch_bounds__(THREADS) void ldbp_fwd_batch_kernel(const cx_t<R>* x, cx_t<R>* y, cx_t<R>* tmp,
                                                                 const BatchWave* __restrict__ waves,
                                                                 const BatchStep* __restrict__ steps,
                                                                 const BatchItem* __restrict__ items, int32_t work,
                                                                 const cx_t<R>* __restrict__ taps,
                                                                 const R* __restrict__ c, int32_t sym) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  V* b0 = reinterpret_cast<V*>(smem);
  V* b1 = b0 + static_cast<size_t>(work + RB) * NPOL;
  const BatchItem it = items[blockIdx.x];
  const BatchWave w = waves[it.wave];
  const int t0 = it.tile * w.tile_len;
  const int Lw = min(w.tile_len, w.n - t0);
  const int H = w.halo;
  const int W0 = Lw + 2 * H;
  const V* xw = (w.src == 0 ? x : w.src == 1 ? static_cast<const V*>(y) : static_cast<const V*>(tmp)) +
                (w.src == 2 ? w.toff : w.off) * NPOL;
  V* yw = (w.dst == 1 ? y : tmp) + (w.dst == 2 ? w.toff : w.off) * NPOL;
  load_tile<R, NPOL, THREADS>(xw, b0, w.n, t0, H, W0, w.wrap);
  __syncthreads();
  int lo = 0;
  for (int s = 0; s < w.nstep; ++s) {
    const BatchStep st = steps[w.step0 + s];
    lo += st.K;
    const R coef = c[st.cidx] * phase_coef_scale<R>();
    fir_kerr_dispatch<R, NPOL, RB, THREADS>(b0, b1, lo, W0 - lo, st.K, taps + st.tapoff, coef, sym != 0);
    __syncthreads();
    V* t = b0;
    b0 = b1;
    b1 = t;
  }
  for (int j = threadIdx.x; j < Lw; j += THREADS)
#pragma unroll
    for (int p = 0; p < NPOL; ++p) yw[static_cast<int64_t>(t0 + j) * NPOL + p] = b0[(H + j) * NPOL + p];
}

}  // namespace ldbp

struct ldbp_batch_plan {
  int32_t dtype, npol, nwave, rb, chunks, work, sym;
  int64_t total_samples, total_sample_steps, total_taps, total_steps;
  int32_t nitems;
  std::vector<int32_t> level_items;   // items of launch g: [level_items[g], level_items[g + 1])
  ldbp::BatchWave* d_waves = nullptr;
  ldbp::BatchStep* d_steps = nullptr;
  ldbp::BatchItem* d_items = nullptr;
  void* d_tmp = nullptr;              // intermediate signal of the waveforms run in several passes
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_taps = nullptr;
  const void* g_c = nullptr;
  const void* g_x = nullptr;
  void* g_y = nullptr;
};

namespace ldbp {

template <typename R, int NPOL, int RB>
static int launch_batch_t(const ldbp_batch_plan* P, const void* taps, const void* c, const void* x, void* y,
                          hipStream_t s) {
  constexpr int THREADS = 256;
  const size_t lds = 2 * static_cast<size_t>(P->work + RB) * NPOL * sizeof(cx_t<R>);
  auto kern = ldbp_fwd_batch_kernel<R, NPOL, RB, THREADS>;
  if (lds > 65536)
    LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  // one launch per pass level: waveforms run in several passes have their later step groups in later
  // launches (each reads what the previous launch wrote)
  for (size_t g = 0; g + 1 < P->level_items.size(); ++g) {
    const int32_t i0 = P->level_items[g], i1 = P->level_items[g + 1];
    if (i1 <= i0) continue;
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(i1 - i0)), dim3(THREADS), lds, s,
                       static_cast<const cx_t<R>*>(x), static_cast<cx_t<R>*>(y), static_cast<cx_t<R>*>(P->d_tmp),
                       P->d_waves, P->d_steps, P->d_items + i0, P->work, static_cast<const cx_t<R>*>(taps),
                       static_cast<const R*>(c), P->sym);
    LDBP_HIP_CHECK(hipGetLastError());
  }
  return LDBP_OK;
}

static int launch_batch(const ldbp_batch_plan* P, const void* taps, const void* c, const void* x, void* y,
                        hipStream_t s) {
#define LDBP_BATCH_LAUNCH(R, NP, B) \
  if (P->npol == NP && P->rb == B) return launch_batch_t<R, NP, B>(P, taps, c, x, y, s);
  if (P->dtype == LDBP_C64) {
    LDBP_BATCH_LAUNCH(float, 1, 7) LDBP_BATCH_LAUNCH(float, 1, 8) LDBP_BATCH_LAUNCH(float, 1, 9)
    LDBP_BATCH_LAUNCH(float, 2, 3) LDBP_BATCH_LAUNCH(float, 2, 4) LDBP_BATCH_LAUNCH(float, 2, 5)
  } else {
    LDBP_BATCH_LAUNCH(double, 1, 3) LDBP_BATCH_LAUNCH(double, 1, 4)
    LDBP_BATCH_LAUNCH(double, 2, 1) LDBP_BATCH_LAUNCH(double, 2, 2)
  }
#undef LDBP_BATCH_LAUNCH
  return fail(LDBP_EUNSUPPORTED, "outputs per thread %d not available", P->rb);
}

static void free_plan(ldbp_batch_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->d_waves) (void)hipFree(P->d_waves);
  if (P->d_steps) (void)hipFree(P->d_steps);
  if (P->d_items) (void)hipFree(P->d_items);
  if (P->d_tmp) (void)hipFree(P->d_tmp);
  delete P;
}

}  // namespace ldbp

using namespace ldbp;

extern "C" int ldbp_batch_plan_create(int32_t dtype, int32_t npol, int32_t nwave, const int64_t* wave_len,
                                      const int32_t* wave_nstep, const int32_t* step_ntap, const ldbp_plan* plan,
                                      ldbp_batch_plan** out) {
  if (!out) return fail(LDBP_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype %d invalid", dtype);
  if (npol != 1 && npol != 2) return fail(LDBP_EUNSUPPORTED, "npol %d not supported", npol);
  if (nwave < 1 || !wave_len || !wave_nstep || !step_ntap) return fail(LDBP_EINVAL, "empty batch or NULL tables");
  const int rb = (plan && plan->outputs_per_thread > 0) ? plan->outputs_per_thread : fwd_rb_default(dtype, npol);
  if (!fwd_rb_supported(dtype, npol, rb)) return fail(LDBP_EUNSUPPORTED, "outputs_per_thread %d not available", rb);
  const int chunk = fwd_chunk(dtype, npol, rb);
  // per waveform: its steps (the step table) and total halo
  struct WaveIn {
    int64_t off;
    int32_t n, nstep, step0, halo;
  };
  std::vector<WaveIn> win(nwave);
  std::vector<BatchStep> steps;
  int64_t off = 0, tapoff = 0, cidx = 0, ss = 0;
  int maxh = 0;
  for (int b = 0; b < nwave; ++b) {
    if (wave_len[b] < 1 || wave_len[b] > (int64_t(1) << 30)) return fail(LDBP_EINVAL, "wave_len[%d] invalid", b);
    if (wave_nstep[b] < 1) return fail(LDBP_EINVAL, "wave_nstep[%d] < 1", b);
    WaveIn& w = win[b];
    w.off = off;
    w.n = static_cast<int32_t>(wave_len[b]);
    w.nstep = wave_nstep[b];
    w.step0 = static_cast<int32_t>(steps.size());
    int h = 0;
    for (int s = 0; s < w.nstep; ++s) {
      const int t = step_ntap[cidx];
      if (t < 1 || t > LDBP_MAX_TAPS || t % 2 == 0) return fail(LDBP_EINVAL, "step tap count %d invalid", t);
      steps.push_back(BatchStep{(t - 1) / 2, static_cast<int32_t>(tapoff), static_cast<int32_t>(cidx), 0});
      h += (t - 1) / 2;
      tapoff += t;
      ++cidx;
    }
    w.halo = h;
    maxh = std::max(maxh, h);
    off += w.n;
    ss += static_cast<int64_t>(w.n) * w.nstep;
  }
  // LDS work size: enough chunks that the longest halo leaves at least half a chunk of tile, within
  // the largest allocation
  int chunks = (plan && plan->chunks > 0) ? plan->chunks : 1;
  while (chunks * chunk - 2 * maxh < chunk / 2 && fwd_lds_bytes(dtype, npol, rb, chunks + 1) <= 160 * 1024) ++chunks;
  if (fwd_lds_bytes(dtype, npol, rb, chunks) > 160 * 1024)
    return fail(LDBP_EUNSUPPORTED, "%d LDS chunks exceed the workgroup's LDS", chunks);
  const int work = chunks * chunk;
  // A waveform whose halo still leaves less than half a chunk of tile runs in several passes: its steps
  // in consecutive groups of halo at most hseg, each group a launch after the previous one, the
  // intermediate signal alternating between y and the plan's buffer so that the last group writes y.
  const int hseg = (work - chunk / 2) / 2;
  std::vector<BatchWave> waves;
  std::vector<int32_t> level;   // pass index of each entry within its waveform
  int64_t toff = 0;
  int nlev = 1;
  for (int b = 0; b < nwave; ++b) {
    const WaveIn& w = win[b];
    std::vector<std::pair<int32_t, int32_t>> groups;   // (first step, steps)
    if (w.halo <= hseg) {
      groups.emplace_back(0, w.nstep);
    } else {
      int s0 = 0, h = 0;
      for (int s = 0; s < w.nstep; ++s) {
        const int K = steps[w.step0 + s].K;
        if (h + K > hseg && s > s0) {
          groups.emplace_back(s0, s - s0);
          s0 = s;
          h = 0;
        }
        h += K;
      }
      groups.emplace_back(s0, w.nstep - s0);
    }
    const int G = static_cast<int>(groups.size());
    nlev = std::max(nlev, G);
    for (int g = 0; g < G; ++g) {
      BatchWave e{};
      e.off = w.off;
      e.toff = toff;
      e.n = w.n;
      e.step0 = w.step0 + groups[g].first;
      e.nstep = groups[g].second;
      int h = 0;
      for (int s = 0; s < e.nstep; ++s) h += steps[e.step0 + s].K;
      e.halo = h;
      e.wrap = h >= w.n ? 1 : 0;
      e.tile_len = work - 2 * h;
      if (e.tile_len < 1) return fail(LDBP_EUNSUPPORTED, "a pass's halo (%d samples) does not fit in LDS", h);
      const int out_buf = ((G - 1 - g) % 2 == 0) ? 1 : 2;
      e.dst = out_buf;
      e.src = g == 0 ? 0 : (((G - g) % 2 == 0) ? 1 : 2);
      waves.push_back(e);
      level.push_back(g);
    }
    if (G > 1) toff += w.n;
  }
  std::vector<BatchItem> sorted;
  std::vector<int32_t> level_items(1, 0);
  for (int g = 0; g < nlev; ++g) {
    std::vector<BatchItem> items;
    std::vector<double> cost;
    for (size_t e = 0; e < waves.size(); ++e) {
      if (level[e] != g) continue;
      const BatchWave& w = waves[e];
      const int nt = (w.n + w.tile_len - 1) / w.tile_len;
      double per_step = 0;
      for (int s = 0; s < w.nstep; ++s) per_step += 2 * steps[w.step0 + s].K + 1 + 8;
      for (int t = 0; t < nt; ++t) {
        items.push_back(BatchItem{static_cast<int32_t>(e), t});
        cost.push_back(per_step * work);
      }
    }
    std::vector<size_t> order(items.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    for (size_t i = 0; i < order.size(); ++i) sorted.push_back(items[order[i]]);
    if (sorted.size() > 0x7fffffffu) return fail(LDBP_EUNSUPPORTED, "too many work items");
    level_items.push_back(static_cast<int32_t>(sorted.size()));
  }

  auto* P = new ldbp_batch_plan();
  P->dtype = dtype;
  P->npol = npol;
  P->nwave = nwave;
  P->rb = rb;
  P->chunks = chunks;
  P->work = work;
  P->sym = (plan && (plan->flags & LDBP_PLAN_SYMMETRIC)) ? 1 : 0;
  P->total_samples = off;
  P->total_sample_steps = ss;
  P->total_taps = tapoff;
  P->total_steps = cidx;
  P->nitems = static_cast<int32_t>(sorted.size());
  P->level_items = level_items;
  hipError_t e = hipGetDevice(&P->device);
  if (e == hipSuccess && toff > 0)
    e = hipMalloc(&P->d_tmp, static_cast<size_t>(toff) * npol * cx_size(dtype));
  if (e == hipSuccess) e = hipMalloc(&P->d_waves, waves.size() * sizeof(BatchWave));
  if (e == hipSuccess) e = hipMalloc(&P->d_steps, std::max<size_t>(steps.size(), 1) * sizeof(BatchStep));
  if (e == hipSuccess) e = hipMalloc(&P->d_items, sorted.size() * sizeof(BatchItem));
  if (e == hipSuccess) e = hipMemcpy(P->d_waves, waves.data(), waves.size() * sizeof(BatchWave), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(P->d_steps, steps.data(), steps.size() * sizeof(BatchStep), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(P->d_items, sorted.data(), sorted.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(P);
    return fail(LDBP_EHIP, "batch plan tables: %s", hipGetErrorString(e));
  }
  *out = P;
  return LDBP_OK;
}

extern "C" int ldbp_batch_plan_destroy(ldbp_batch_plan* plan) {
  free_plan(plan);
  return LDBP_OK;
}

extern "C" int ldbp_batch_plan_info(const ldbp_batch_plan* P, int64_t* total_samples, int64_t* total_sample_steps,
                                    int64_t* total_taps, int64_t* total_steps, int32_t* nitems, int32_t* work) {
  if (!P) return fail(LDBP_EINVAL, "plan is NULL");
  if (total_samples) *total_samples = P->total_samples;
  if (total_sample_steps) *total_sample_steps = P->total_sample_steps;
  if (total_taps) *total_taps = P->total_taps;
  if (total_steps) *total_steps = P->total_steps;
  if (nitems) *nitems = P->nitems;
  if (work) *work = P->work;
  return LDBP_OK;
}

static int check_batch_args(const ldbp_batch_plan* P, const void* taps, const void* c, const void* x, void* y) {
  if (!P) return fail(LDBP_EINVAL, "plan is NULL");
  if (!taps || !c || !x || !y) return fail(LDBP_EINVAL, "taps, c, x and y must be non-NULL");
  if (!aligned16(taps) || !aligned16(x) || !aligned16(y)) return fail(LDBP_EINVAL, "arrays must be 16-byte aligned");
  const size_t wb = static_cast<size_t>(P->total_samples) * P->npol * cx_size(P->dtype);
  if (overlaps(x, wb, y, wb)) return fail(LDBP_EINVAL, "x and y overlap");
  return LDBP_OK;
}

extern "C" int ldbp_batch_forward(const ldbp_batch_plan* P, const void* taps, const void* c, const void* x, void* y,
                                  void* stream) {
  int st = check_batch_args(P, taps, c, x, y);
  if (st) return st;
  return launch_batch(P, taps, c, x, y, static_cast<hipStream_t>(stream));
}

extern "C" int ldbp_batch_forward_graph(ldbp_batch_plan* P, const void* taps, const void* c, const void* x, void* y,
                                        void* stream) {
  int st = check_batch_args(P, taps, c, x, y);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!P->exec || P->g_taps != taps || P->g_c != c || P->g_x != x || P->g_y != y) {
    if (P->exec) {
      (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
    }
    if (P->graph) {
      (void)hipGraphDestroy(P->graph);
      P->graph = nullptr;
    }
    hipStream_t cap;
    LDBP_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const int lst = launch_batch(P, taps, c, x, y, cap);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cap, &g);
      if (lst != LDBP_OK) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cap);
        return lst;
      }
      e = e2;
      if (e == hipSuccess) {
        P->graph = g;
        e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
      }
    }
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(LDBP_EHIP, "graph capture: %s", hipGetErrorString(e));
    P->g_taps = taps;
    P->g_c = c;
    P->g_x = x;
    P->g_y = y;
  }
  LDBP_HIP_CHECK(hipGraphLaunch(P->exec, s));
  return LDBP_OK;
}
