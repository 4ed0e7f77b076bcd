// C ABI of the LDBP and generalised-ESSM forward (periodic, checkpointed, aperiodic) and backward:
// validation, planning, pass sequencing and the batch split over a second stream.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "common.h"
#include "ldbp_kernels.h"

namespace ldbp {

constexpr size_t kMaxLdsBytes = 160 * 1024;

static size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Guard mode (LDBP_PLAN_GUARD): the non-finite flag takes the last 256 bytes of the forward's workspace.
constexpr size_t kGuardBytes = 256;

struct ModelArgs {
  int32_t dtype, npol;
  int64_t nwave, n;
  int32_t nstep;
  const int32_t* ntap;
  const int32_t* nl_ntap = nullptr;  // filtered nonlinear steps (generalised ESSM): real filter lengths

  int kap(int i) const { return nl_ntap ? (nl_ntap[i] - 1) / 2 : 0; }
  bool filtered() const { return nl_ntap != nullptr; }
};

static int check_model(const ModelArgs& m) {
  if (m.dtype != LDBP_C64 && m.dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype %d is not LDBP_C64/LDBP_C128", m.dtype);
  if (m.npol != 1 && m.npol != 2) return fail(LDBP_EUNSUPPORTED, "npol %d not supported (1 or 2)", m.npol);
  if (m.nwave < 1) return fail(LDBP_EINVAL, "nwave %lld < 1", (long long)m.nwave);
  if (m.n < 1 || m.n > (1LL << 30)) return fail(LDBP_EINVAL, "n %lld outside [1, 2^30]", (long long)m.n);
  if (m.nstep < 1) return fail(LDBP_EINVAL, "nstep %d < 1", m.nstep);
  if (!m.ntap) return fail(LDBP_EINVAL, "ntap is NULL");
  for (int i = 0; i < m.nstep; ++i) {
    const int t = m.ntap[i];
    if (t < 1 || t > LDBP_MAX_TAPS || (t % 2) == 0)
      return fail(LDBP_EINVAL, "ntap[%d] = %d must be odd and in [1, %d]", i, t, LDBP_MAX_TAPS);
    if (m.nl_ntap) {
      const int e = m.nl_ntap[i];
      if (e < 1 || e > LDBP_MAX_NL_TAPS || (e % 2) == 0)
        return fail(LDBP_EINVAL, "nl_ntap[%d] = %d must be odd and in [1, %d]", i, e, LDBP_MAX_NL_TAPS);
    }
  }
  return LDBP_OK;
}

// A second stream per host thread, device and caller stream, with the two events that fork it from
// the caller's stream and join it back.  Created on first use and kept until the process ends.
// Keyed by the caller's stream so that calls on different streams stay independent of each other.
struct SideStream {
  int dev = -1;
  hipStream_t caller = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr size_t kMaxSideStreams = 16;  // per host thread; further caller streams run on one stream

// The side stream for work forked from `caller`, or NULL when the call should stay on one stream:
// the caller's stream is being captured, belongs to another device than the current one, the
// thread already keeps kMaxSideStreams of them, or a runtime call fails (its error is cleared; the
// work then simply runs on one stream).
static SideStream* side_stream(hipStream_t caller) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(caller, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (caller) {
    hipDevice_t sd = -1;
    if (hipStreamGetDevice(caller, &sd) != hipSuccess || sd != cur) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  thread_local std::vector<SideStream> sides;
  for (auto& x : sides)
    if (x.dev == cur && x.caller == caller) return x.s ? &x : nullptr;
  if (sides.size() >= kMaxSideStreams) return nullptr;
  SideStream x;
  x.dev = cur;
  x.caller = caller;
  if (hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&x.join, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    x.s = nullptr;  // remembered: this caller stream keeps to one stream
  }
  sides.push_back(x);
  return x.s ? &sides.back() : nullptr;
}

// Runs the launches run(k, w0, w1, stream), k = 0 .. nstep - 1, over the waveforms of the batch: with
// split, waveforms [h, nwave) on the side stream (forked from s, joined back into s) and [0, h) on s,
// h = ceil(nwave / 2); otherwise all of them on s.  The two halves touch disjoint waveforms, so the
// kernels of one fill the other's ramp-up and drain at every launch boundary.  The halves' launches are
// enqueued alternately (launch k of the first half, then launch k of the second): the second half then
// starts with the first instead of after the host has enqueued every launch of the first, which for
// the 32 launches of a two-polarisation backward left it 7 launches behind.
template <typename F>
static int over_halves(hipStream_t s, int64_t nwave, bool split, size_t nstep, F&& run) {
  SideStream* side = (split && nwave >= 2) ? side_stream(s) : nullptr;
  if (!side) {
    for (size_t k = 0; k < nstep; ++k) {
      const int st = run(k, int64_t(0), nwave, s);
      if (st) return st;
    }
    return LDBP_OK;
  }
  const int64_t h = (nwave + 1) / 2;
  LDBP_HIP_CHECK(hipEventRecord(side->fork, s));
  LDBP_HIP_CHECK(hipStreamWaitEvent(side->s, side->fork, 0));
  int st = LDBP_OK;
  for (size_t k = 0; k < nstep && !st; ++k) {
    st = run(k, int64_t(0), h, s);
    if (!st) st = run(k, h, nwave, side->s);
  }
  // join even after a failed launch, so that later work on s stays ordered after everything enqueued
  LDBP_HIP_CHECK(hipEventRecord(side->join, side->s));
  LDBP_HIP_CHECK(hipStreamWaitEvent(s, side->join, 0));
  return st;
}

// The split pays when a call has several launches of at least two workgroups per compute unit.
static bool worth_splitting(const ldbp_plan* plan, size_t launches, int64_t blocks_per_launch) {
  if (plan && (plan->flags & LDBP_PLAN_ONE_STREAM)) return false;
  return launches >= 2 && blocks_per_launch >= 512;
}

static int max_chunks(int dtype, int npol, int rb, bool filtered = false) {
  int c = 1;
  while (fwd_lds_bytes(dtype, npol, rb, c + 1, filtered) <= kMaxLdsBytes) ++c;
  return c;
}

// Default LDS work size: the most chunks that still let three workgroups share a compute unit's LDS.
// Larger tiles cut the halo recomputed per output and the passes over HBM, but below three resident
// workgroups the memory latency is no longer hidden: with 5-tap filters on two polarisations
// (3 outputs per thread) 2 chunks run the checkpointing forward in 1.12 ms against 1.25 ms for 1 and
// 1.20 ms for 3; with 15 taps on one polarisation (7 outputs per thread) 1 chunk beats 2 by 20%.
static int default_chunks(int dtype, int npol, int rb, bool filtered) {
  int c = 1;
  while (3 * fwd_lds_bytes(dtype, npol, rb, c + 1, filtered) <= kMaxLdsBytes) ++c;
  return c;
}

// Splits the l steps into passes.  With a checkpoint interval the passes are
// exactly the checkpoint blocks (the backward's unit; the forward groups them, see
// make_block_plan); otherwise each pass takes steps while twice its halo stays within
// 1/8 of the LDS work size (or a fixed S from the plan), and the steps are then spread
// evenly over that many passes (no short last pass paying a full read and write of the signal).
struct PassPlan {
  std::vector<PassTable> passes;
  int chunks;
  int rb;   // outputs per thread
  int sym;  // folded evaluation of symmetric filters
};

static int make_plan(const ModelArgs& m, int32_t ckpt_every, const ldbp_plan* plan, PassPlan& out) {
  const int rb = (plan && plan->outputs_per_thread > 0) ? plan->outputs_per_thread : fwd_rb_default(m.dtype, m.npol);
  if (!fwd_rb_supported(m.dtype, m.npol, rb))
    return fail(LDBP_EUNSUPPORTED, "outputs_per_thread %d not available for this dtype/npol", rb);
  out.rb = rb;
  out.sym = (plan && (plan->flags & LDBP_PLAN_SYMMETRIC)) ? 1 : 0;
  const int chunk = fwd_chunk(m.dtype, m.npol, rb);
  int chunks = (plan && plan->chunks > 0) ? plan->chunks : default_chunks(m.dtype, m.npol, rb, m.filtered());
  const int cmax = max_chunks(m.dtype, m.npol, rb, m.filtered());
  if (chunks > cmax) return fail(LDBP_EINVAL, "plan chunks %d exceeds the LDS limit (%d)", chunks, cmax);
  const int fixed_s = ckpt_every > 0 ? ckpt_every : ((plan && plan->steps_per_pass > 0) ? plan->steps_per_pass : 0);
  if (fixed_s > LDBP_MAX_STEPS_PER_PASS)
    return fail(LDBP_EINVAL, "steps per pass %d exceeds %d", fixed_s, LDBP_MAX_STEPS_PER_PASS);

  std::vector<int32_t> tapoff(m.nstep), etaoff(m.nstep);
  int32_t acc = 0, eacc = 0;
  for (int i = 0; i < m.nstep; ++i) {
    tapoff[i] = acc;
    acc += m.ntap[i];
    etaoff[i] = eacc;
    eacc += m.nl_ntap ? m.nl_ntap[i] : 1;
  }
  // greedy split, at most `cap` steps per pass
  auto split = [&](int cap) {
    out.passes.clear();
    int s = 0;
    while (s < m.nstep) {
      PassTable pt{};
      pt.c0 = s;
      int h = 0;
      int cnt = 0;
      while (s + cnt < m.nstep && cnt < cap) {
        const int kf = (m.ntap[s + cnt] - 1) / 2;
        const int k = kf + m.kap(s + cnt);  // halo of the step: FIR half-length plus power-filter half-length
        if (fixed_s == 0 && cnt > 0 && 2 * (h + k) * 8 > chunks * chunk) break;
        pt.K[cnt] = kf;
        pt.tapoff[cnt] = tapoff[s + cnt];
        pt.kap[cnt] = m.kap(s + cnt);
        pt.etaoff[cnt] = etaoff[s + cnt];
        h += k;
        ++cnt;
      }
      pt.nstep = cnt;
      pt.halo = h;
      pt.wrap_general = (h >= m.n) ? 1 : 0;
      out.passes.push_back(pt);
      s += cnt;
    }
  };
  split(fixed_s > 0 ? fixed_s : LDBP_MAX_STEPS_PER_PASS);
  if (fixed_s == 0 && out.passes.size() > 1) {
    const int np = static_cast<int>(out.passes.size());
    split((m.nstep + np - 1) / np);
  }
  int max_halo = 0;
  for (const auto& pt : out.passes) max_halo = std::max(max_halo, pt.halo);
  // Grow the LDS work size when a pass's halo leaves too little room for the tile.
  while (chunks * chunk - 2 * max_halo < chunk / 2 && chunks < cmax) ++chunks;
  if (chunks * chunk - 2 * max_halo < 1)
    return fail(LDBP_EUNSUPPORTED, "halo %d of a %d-step pass does not fit in LDS; use fewer steps per pass",
                max_halo, fixed_s);
  out.chunks = chunks;
  return LDBP_OK;
}

// Passes over steps [0, nrun) made of whole checkpoint blocks of S steps: a pass takes blocks
// while twice its halo stays within 1/8 of the LDS work size, the blocks then spread evenly over
// that many passes (or up to plan->steps_per_pass steps, at least one block), and writes the state
// at each inner block boundary to that block's slot (ckpt_mask).  The pass output itself is the
// next block's slot, or y after the last step.
static int make_block_plan(const ModelArgs& m, int32_t S, int32_t nrun, const ldbp_plan* plan, PassPlan& out) {
  int st = make_plan(m, S, plan, out);  // exact blocks: validates rb, chunks and the per-block halo
  if (st) return st;
  const int chunk = fwd_chunk(m.dtype, m.npol, out.rb);
  const int cmax = max_chunks(m.dtype, m.npol, out.rb, m.filtered());
  const int want = (plan && plan->steps_per_pass > 0) ? std::max<int>(S, plan->steps_per_pass / S * S) : 0;
  std::vector<PassTable> blocks;
  for (const auto& b : out.passes)
    if (b.c0 < nrun) blocks.push_back(b);
  std::vector<PassTable> passes;
  // greedy grouping, at most `cap` blocks per pass
  auto group = [&](size_t cap) {
    passes.clear();
    for (size_t i = 0; i < blocks.size();) {
      PassTable pt = blocks[i];
      pt.ckpt_mask = 0;
      pt.ckpt_every = S;
      size_t j = i + 1;
      while (j < blocks.size() && j - i < cap) {
        const PassTable& b = blocks[j];
        if (pt.nstep + b.nstep > LDBP_MAX_STEPS_PER_PASS) break;
        if (want > 0 ? pt.nstep + b.nstep > want : 2 * (pt.halo + b.halo) * 8 > out.chunks * chunk) break;
        pt.ckpt_mask |= uint64_t(1) << (pt.nstep - 1);  // the end of the pass so far is an inner boundary
        for (int k = 0; k < b.nstep; ++k) {
          pt.K[pt.nstep + k] = b.K[k];
          pt.tapoff[pt.nstep + k] = b.tapoff[k];
          pt.kap[pt.nstep + k] = b.kap[k];
          pt.etaoff[pt.nstep + k] = b.etaoff[k];
        }
        pt.nstep += b.nstep;
        pt.halo += b.halo;
        ++j;
      }
      pt.wrap_general = (pt.halo >= m.n) ? 1 : 0;
      passes.push_back(pt);
      i = j;
    }
  };
  group(blocks.size());
  if (want == 0 && passes.size() > 1) group((blocks.size() + passes.size() - 1) / passes.size());
  int max_halo = 0;
  for (const auto& pt : passes) max_halo = std::max(max_halo, pt.halo);
  int chunks = out.chunks;
  while (chunks * chunk - 2 * max_halo < chunk / 2 && chunks < cmax) ++chunks;
  if (chunks * chunk - 2 * max_halo < 1)
    return fail(LDBP_EUNSUPPORTED, "halo %d of a pass does not fit in LDS; use fewer steps per pass", max_halo);
  out.chunks = chunks;
  out.passes = passes;
  return LDBP_OK;
}

// Pass i of a block plan over waveforms [w0, w1): its input is x (i = 0) or the previous pass's output;
// its output is the next block's checkpoint slot, or `last` (y, or the last slot) after the final pass;
// inner block inputs b >= 1 go to slot b - 1 of ckpt.  Pointers are those of the whole batch.
static int launch_block_pass(const ModelArgs& m, const PassPlan& pp, size_t i, const void* taps, const void* c,
                             const void* x, void* last, void* ckpt, int32_t S, hipStream_t s, const void* eta,
                             int64_t w0, int64_t w1, int32_t* nonfinite = nullptr) {
  const size_t wave_bytes = static_cast<size_t>(m.nwave) * m.n * m.npol * cx_size(m.dtype);
  const size_t w_off = static_cast<size_t>(w0) * m.n * m.npol * cx_size(m.dtype);
  const int64_t slot_elems = m.nwave * m.n * m.npol;
  auto pass_out = [&](size_t j) {
    const PassTable& pt = pp.passes[j];
    return ((j + 1 == pp.passes.size()) ? static_cast<char*>(last)
                                        : static_cast<char*>(ckpt) + ((pt.c0 + pt.nstep) / S - 1) * wave_bytes) + w_off;
  };
  const void* in = i == 0 ? static_cast<const char*>(x) + w_off : pass_out(i - 1);
  const bool final_pass = i + 1 == pp.passes.size();
  return launch_fwd_pass(m.dtype, m.npol, pp.rb, in, pass_out(i), w1 - w0, static_cast<int32_t>(m.n), pp.chunks,
                         pp.passes[i], taps, c, pp.sym, ckpt ? static_cast<char*>(ckpt) + w_off : nullptr, s, eta,
                         slot_elems, nullptr, final_pass ? nonfinite : nullptr);
}

// Workgroups of one forward launch over the batch (the pass with the largest halo has the most tiles).
static int64_t fwd_blocks(const ModelArgs& m, const PassPlan& pp) {
  int32_t halo = 0;
  for (const auto& pt : pp.passes) halo = std::max(halo, pt.halo);
  const int64_t tile = std::max<int64_t>(1, int64_t(pp.chunks) * fwd_chunk(m.dtype, m.npol, pp.rb) - 2 * halo);
  return m.nwave * ((m.n + tile - 1) / tile);
}

}  // namespace ldbp

using namespace ldbp;

namespace ldbp {

static int forward_ws_impl(const ModelArgs& m, const void* ckpt, const ldbp_plan* plan, size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  int st = check_model(m);
  if (st) return st;
  const size_t guard = (plan && (plan->flags & LDBP_PLAN_GUARD)) ? kGuardBytes : 0;
  if (ckpt) {
    *bytes = guard;
    return LDBP_OK;
  }
  PassPlan pp;
  st = make_plan(m, 0, plan, pp);
  if (st) return st;
  const size_t wave_bytes = static_cast<size_t>(m.nwave) * m.n * m.npol * cx_size(m.dtype);
  *bytes = pp.passes.size() > 1 ? (guard ? align256(wave_bytes) + guard : wave_bytes) : guard;
  return LDBP_OK;
}

__global__ void clear_flag_kernel(int32_t* flag) { *flag = 0; }

// Guard mode: the flag the last pass raises is copied to the host after the whole call (both halves
// of a split batch have been joined into s), which synchronises the stream.
static int guard_result(int32_t* flag, hipStream_t s) {
  int32_t h = 0;
  LDBP_HIP_CHECK(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
  LDBP_HIP_CHECK(hipStreamSynchronize(s));
  if (h) return fail(LDBP_ENONFINITE, "the forward output holds a NaN or an infinity (guard mode)");
  return LDBP_OK;
}

// The forward of LDBP (eta == NULL) and of the generalised ESSM (eta: packed real filters, m.nl_ntap).
static int forward_impl(const ModelArgs& m, const void* taps, const void* c, const void* eta, const void* x, void* y,
                        void* ckpt, int32_t ckpt_every, const ldbp_plan* plan, void* ws, size_t ws_bytes,
                        void* stream) {
  int st = check_model(m);
  if (st) return st;
  if (!taps || !c || !x || !y) return fail(LDBP_EINVAL, "taps, c, x and y must be non-NULL");
  if (m.filtered() && !eta) return fail(LDBP_EINVAL, "eta must be non-NULL");
  if (!aligned16(taps) || !aligned16(x) || !aligned16(y)) return fail(LDBP_EINVAL, "taps, x and y must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(c) % real_size(m.dtype)) return fail(LDBP_EINVAL, "c is not aligned to its real type");
  if (eta && reinterpret_cast<uintptr_t>(eta) % real_size(m.dtype))
    return fail(LDBP_EINVAL, "eta is not aligned to its real type");
  const size_t wave_bytes = static_cast<size_t>(m.nwave) * m.n * m.npol * cx_size(m.dtype);
  if (overlaps(x, wave_bytes, y, wave_bytes)) return fail(LDBP_EINVAL, "x and y overlap");
  if (ckpt) {
    if (ckpt_every < 1 || ckpt_every > LDBP_MAX_STEPS_PER_PASS)
      return fail(LDBP_EINVAL, "ckpt_every %d outside [1, %d]", ckpt_every, LDBP_MAX_STEPS_PER_PASS);
    if (!aligned16(ckpt)) return fail(LDBP_EINVAL, "ckpt must be 16-byte aligned");
    const int64_t nslot = (m.nstep + ckpt_every - 1) / ckpt_every - 1;
    if (nslot > 0 && (overlaps(ckpt, nslot * wave_bytes, x, wave_bytes) || overlaps(ckpt, nslot * wave_bytes, y, wave_bytes)))
      return fail(LDBP_EINVAL, "ckpt overlaps x or y");
  }
  if (plan && (plan->flags & ~(LDBP_PLAN_SYMMETRIC | LDBP_PLAN_ONE_STREAM | LDBP_PLAN_GUARD)))
    return fail(LDBP_EINVAL, "plan flags 0x%x: unknown bits", plan->flags);
  const bool guard = plan && (plan->flags & LDBP_PLAN_GUARD);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* e = m.filtered() ? eta : nullptr;
  PassPlan pp;
  if (ckpt) st = make_block_plan(m, ckpt_every, m.nstep, plan, pp);
  else st = make_plan(m, 0, plan, pp);
  if (st) return st;
  const size_t np = pp.passes.size();
  // ping-pong buffer of a multi-pass forward, followed (guard mode) by the flag at a 256-byte boundary
  const size_t inter = (!ckpt && np > 1) ? (guard ? align256(wave_bytes) : wave_bytes) : 0;
  const size_t need = inter + (guard ? kGuardBytes : 0);
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(LDBP_EWORKSPACE, "workspace of %zu bytes required, %zu given", need, ws ? ws_bytes : 0);
    if (!aligned16(ws)) return fail(LDBP_EINVAL, "ws must be 16-byte aligned");
    if (overlaps(ws, need, x, wave_bytes) || overlaps(ws, need, y, wave_bytes))
      return fail(LDBP_EINVAL, "workspace overlaps x or y");
    if (ckpt) {
      const int64_t nslot = (m.nstep + ckpt_every - 1) / ckpt_every - 1;
      if (nslot > 0 && overlaps(ws, need, ckpt, nslot * wave_bytes)) return fail(LDBP_EINVAL, "workspace overlaps ckpt");
    }
  }
  int32_t* flag = guard ? reinterpret_cast<int32_t*>(static_cast<char*>(ws) + inter) : nullptr;
  if (flag) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    LDBP_HIP_CHECK(hipGetLastError());
  }
  if (ckpt) {
    st = over_halves(s, m.nwave, worth_splitting(plan, np, fwd_blocks(m, pp)), np,
                     [&](size_t i, int64_t w0, int64_t w1, hipStream_t ss) {
                       return launch_block_pass(m, pp, i, taps, c, x, y, ckpt, ckpt_every, ss, e, w0, w1, flag);
                     });
    return (st || !flag) ? st : guard_result(flag, s);
  }
  const size_t wave_elem_bytes = static_cast<size_t>(m.n) * m.npol * cx_size(m.dtype);
  st = over_halves(s, m.nwave, worth_splitting(plan, np, fwd_blocks(m, pp)), np,
                   [&](size_t i, int64_t w0, int64_t w1, hipStream_t ss) {
                     const size_t off = static_cast<size_t>(w0) * wave_elem_bytes;
                     // ping-pong that ends in y: pass i writes y when np - 1 - i is even, ws otherwise
                     auto out_of = [&](size_t j) { return static_cast<char*>(((np - 1 - j) % 2 == 0) ? y : ws) + off; };
                     const void* in = i == 0 ? static_cast<const char*>(x) + off : out_of(i - 1);
                     return launch_fwd_pass(m.dtype, m.npol, pp.rb, in, out_of(i), w1 - w0, static_cast<int32_t>(m.n),
                                            pp.chunks, pp.passes[i], taps, c, pp.sym, nullptr, ss, e, 0, nullptr,
                                            i + 1 == np ? flag : nullptr);
                   });
  return (st || !flag) ? st : guard_result(flag, s);
}

// Aperiodic forward: the passes of the periodic forward on a working circle of nw samples per
// waveform (n + 2P with zero margins, or n for VALID), the first pass reading x through an EdgeMap
// and the last one storing only the nout output positions.  P = sum (K_i + kappa_i) bounds the
// dependence of an output, so no value that reaches a stored output ever wraps around the circle.
struct AperGeom {
  int64_t P, nw, nout;
  size_t buf_bytes;  // one intermediate buffer (nwave working waveforms)
  int nbuf;          // intermediate buffers: 0 (one pass), 1 (two) or 2 (ping-pong)
};

static int aperiodic_geom(const ModelArgs& m, int32_t edge, const ldbp_plan* plan, PassPlan& pp, AperGeom& g) {
  if (edge != LDBP_EDGE_ZERO && edge != LDBP_EDGE_VALID)
    return fail(LDBP_EINVAL, "edge %d is not LDBP_EDGE_ZERO/LDBP_EDGE_VALID", edge);
  g.P = 0;
  for (int i = 0; i < m.nstep; ++i) g.P += (m.ntap[i] - 1) / 2 + m.kap(i);
  if (edge == LDBP_EDGE_VALID) {
    if (m.n <= 2 * g.P)
      return fail(LDBP_EINVAL, "n = %lld leaves no valid output (2P = %lld)", (long long)m.n, (long long)(2 * g.P));
    g.nw = m.n;
    g.nout = m.n - 2 * g.P;
  } else {
    g.nw = m.n + 2 * g.P;
    g.nout = m.n;
    if (g.nw > (1LL << 30)) return fail(LDBP_EUNSUPPORTED, "n + 2P = %lld exceeds 2^30", (long long)g.nw);
  }
  ModelArgs mw = m;
  mw.n = g.nw;
  const int st = make_plan(mw, 0, plan, pp);
  if (st) return st;
  const size_t np = pp.passes.size();
  g.nbuf = np >= 3 ? 2 : (np == 2 ? 1 : 0);
  g.buf_bytes = align256(static_cast<size_t>(m.nwave) * g.nw * m.npol * cx_size(m.dtype));
  return LDBP_OK;
}

static int aperiodic_ws_impl(const ModelArgs& m, int32_t edge, const ldbp_plan* plan, size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  int st = check_model(m);
  if (st) return st;
  PassPlan pp;
  AperGeom g;
  st = aperiodic_geom(m, edge, plan, pp, g);
  if (st) return st;
  *bytes = g.nbuf * g.buf_bytes;
  return LDBP_OK;
}

static int aperiodic_impl(const ModelArgs& m, const void* taps, const void* c, const void* eta, const void* x,
                          void* y, int32_t edge, const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  int st = check_model(m);
  if (st) return st;
  if (!taps || !c || !x || !y) return fail(LDBP_EINVAL, "taps, c, x and y must be non-NULL");
  if (m.filtered() && !eta) return fail(LDBP_EINVAL, "eta must be non-NULL");
  if (!aligned16(taps) || !aligned16(x) || !aligned16(y)) return fail(LDBP_EINVAL, "taps, x and y must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(c) % real_size(m.dtype)) return fail(LDBP_EINVAL, "c is not aligned to its real type");
  if (eta && reinterpret_cast<uintptr_t>(eta) % real_size(m.dtype))
    return fail(LDBP_EINVAL, "eta is not aligned to its real type");
  if (plan && (plan->flags & ~(LDBP_PLAN_SYMMETRIC | LDBP_PLAN_ONE_STREAM)))
    return fail(LDBP_EINVAL, "plan flags 0x%x: unknown bits", plan->flags);
  PassPlan pp;
  AperGeom g;
  st = aperiodic_geom(m, edge, plan, pp, g);
  if (st) return st;
  const size_t sample_bytes = static_cast<size_t>(m.npol) * cx_size(m.dtype);
  const size_t x_bytes = static_cast<size_t>(m.nwave) * m.n * sample_bytes;
  const size_t y_bytes = static_cast<size_t>(m.nwave) * g.nout * sample_bytes;
  if (overlaps(x, x_bytes, y, y_bytes)) return fail(LDBP_EINVAL, "x and y overlap");
  const size_t need = g.nbuf * g.buf_bytes;
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(LDBP_EWORKSPACE, "workspace of %zu bytes required, %zu given", need, ws ? ws_bytes : 0);
    if (!aligned16(ws)) return fail(LDBP_EINVAL, "ws must be 16-byte aligned");
    if (overlaps(ws, need, x, x_bytes) || overlaps(ws, need, y, y_bytes))
      return fail(LDBP_EINVAL, "workspace overlaps x or y");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* e = m.filtered() ? eta : nullptr;
  const size_t np = pp.passes.size();
  ModelArgs mw = m;
  mw.n = g.nw;
  const int32_t nw = static_cast<int32_t>(g.nw);
  return over_halves(s, m.nwave, worth_splitting(plan, np, fwd_blocks(mw, pp)), np,
                     [&](size_t i, int64_t w0, int64_t w1, hipStream_t ss) {
                       const bool first = i == 0, last = i + 1 == np;
                       EdgeMap em{0, nw, 0, nw};
                       if (first) em.in_len = static_cast<int32_t>(m.n);
                       if (first && edge == LDBP_EDGE_ZERO) em.in_off = static_cast<int32_t>(g.P);
                       if (last) {
                         em.out_off = static_cast<int32_t>(g.P);
                         em.out_len = static_cast<int32_t>(g.nout);
                       }
                       const bool use_em = last || (first && edge == LDBP_EDGE_ZERO);
                       // passes alternate between the two work buffers; the last writes y
                       const char* in = first ? static_cast<const char*>(x) + w0 * m.n * sample_bytes
                                              : static_cast<const char*>(ws) + ((i - 1) % 2) * g.buf_bytes +
                                                    w0 * g.nw * sample_bytes;
                       char* out = last ? static_cast<char*>(y) + w0 * g.nout * sample_bytes
                                        : static_cast<char*>(ws) + (i % 2) * g.buf_bytes + w0 * g.nw * sample_bytes;
                       return launch_fwd_pass(m.dtype, m.npol, pp.rb, in, out, w1 - w0, nw, pp.chunks, pp.passes[i],
                                              taps, c, pp.sym, nullptr, ss, e, 0, use_em ? &em : nullptr);
                     });
}

static int plan_query_impl(const ModelArgs& m, int32_t ckpt_every, const ldbp_plan* plan, int32_t* npasses,
                           int32_t* tile_len, int32_t* max_steps_per_pass) {
  int st = check_model(m);
  if (st) return st;
  if (ckpt_every < 0 || ckpt_every > LDBP_MAX_STEPS_PER_PASS)
    return fail(LDBP_EINVAL, "ckpt_every %d outside [0, %d]", ckpt_every, LDBP_MAX_STEPS_PER_PASS);
  PassPlan pp;
  st = ckpt_every > 0 ? make_block_plan(m, ckpt_every, m.nstep, plan, pp) : make_plan(m, 0, plan, pp);
  if (st) return st;
  int maxs = 0, minlen = 1 << 30;
  for (const auto& pt : pp.passes) {
    maxs = std::max(maxs, pt.nstep);
    minlen = std::min(minlen, pp.chunks * fwd_chunk(m.dtype, m.npol, pp.rb) - 2 * pt.halo);
  }
  if (npasses) *npasses = static_cast<int32_t>(pp.passes.size());
  if (tile_len) *tile_len = minlen;
  if (max_steps_per_pass) *max_steps_per_pass = maxs;
  return LDBP_OK;
}

}  // namespace ldbp

namespace ldbp {

// ---------------------------------------------------------------- forward without allocation
//
// ldbp_forward_noalloc runs ldbp_forward with its workspace (the ping-pong buffer of a multi-pass
// forward and the guard flag) taken from `scratch`, a static device array that every GPU the library
// runs on holds until the process ends.  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device, on the first call with that
// device current.  Every call on a device shares that device's array, so calls that overlap in time
// on one device (other streams, other host threads) race; the guard flag is cleared by a kernel at
// the start of each guarded call, and the ping-pong buffer is fully written before it is read.
static __device__ __align__(256) unsigned char scratch[LDBP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(void** out) {
  int dev = -1;
  LDBP_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LDBP_EUNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LDBP_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LDBP_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LDBP_OK;
}

}  // namespace ldbp

extern "C" int ldbp_forward_noalloc(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                    const int32_t* ntap, const void* taps, const void* c, const void* x, void* y,
                                    void* ckpt, int32_t ckpt_every, const ldbp_plan* plan, void* stream) {
  const ModelArgs m{dtype, npol, nwave, n, nstep, ntap};
  // always one stream: the batch split would create a second stream on first use
  ldbp_plan p{0, 0, 0, LDBP_PLAN_ONE_STREAM};
  if (plan)
    p = ldbp_plan{plan->steps_per_pass, plan->chunks, plan->outputs_per_thread, plan->flags | LDBP_PLAN_ONE_STREAM};
  size_t need = 0;
  int st = forward_ws_impl(m, ckpt, &p, &need);
  if (st) return st;
  if (need > LDBP_NOALLOC_SCRATCH_BYTES)
    return fail(LDBP_EWORKSPACE,
                "ldbp_forward_noalloc needs %zu bytes of scratch; its static scratch holds %zu "
                "(LDBP_NOALLOC_SCRATCH_BYTES): use ldbp_forward with a workspace, or a smaller batch",
                need, static_cast<size_t>(LDBP_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  if (need > 0) {
    st = scratch_address(&ws);
    if (st) return st;
  }
  return forward_impl(m, taps, c, nullptr, x, y, ckpt, ckpt_every, &p, ws,
                      need > 0 ? static_cast<size_t>(LDBP_NOALLOC_SCRATCH_BYTES) : 0, stream);
}

extern "C" int ldbp_forward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                           const int32_t* ntap, const void* ckpt, int32_t ckpt_every,
                                           const ldbp_plan* plan, size_t* bytes) {
  (void)ckpt_every;
  return forward_ws_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap}, ckpt, plan, bytes);
}

extern "C" int ldbp_forward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                            const int32_t* ntap, const void* taps, const void* c, const void* x, void* y,
                            void* ckpt, int32_t ckpt_every, const ldbp_plan* plan, void* ws, size_t ws_bytes,
                            void* stream) {
  return forward_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap}, taps, c, nullptr, x, y, ckpt, ckpt_every, plan,
                      ws, ws_bytes, stream);
}

extern "C" int essm_forward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                           const int32_t* ntap, const int32_t* nl_ntap, const void* ckpt,
                                           int32_t ckpt_every, const ldbp_plan* plan, size_t* bytes) {
  (void)ckpt_every;
  if (!nl_ntap) return fail(LDBP_EINVAL, "nl_ntap is NULL");
  return forward_ws_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, ckpt, plan, bytes);
}

extern "C" int essm_forward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                            const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                            const void* eta, const void* x, void* y, void* ckpt, int32_t ckpt_every,
                            const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  if (!nl_ntap) return fail(LDBP_EINVAL, "nl_ntap is NULL");
  return forward_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, taps, c, eta, x, y, ckpt, ckpt_every,
                      plan, ws, ws_bytes, stream);
}

extern "C" int essm_forward_plan_query(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                       const int32_t* ntap, const int32_t* nl_ntap, int32_t ckpt_every,
                                       const ldbp_plan* plan, int32_t* npasses, int32_t* tile_len,
                                       int32_t* max_steps_per_pass) {
  if (!nl_ntap) return fail(LDBP_EINVAL, "nl_ntap is NULL");
  return plan_query_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, ckpt_every, plan, npasses, tile_len,
                         max_steps_per_pass);
}

// ---------------------------------------------------------------- backward

namespace ldbp {

// Three workgroups per CU.  Two polarisations as well: with the short-filter kernel variants (84
// registers at 5 taps) 53 KiB measured 7% faster than 80 KiB on 8 x 2^20 x 2 (l = 64, 5 taps, 3 steps
// per checkpoint block: 6.42 against 6.94 ms for forward with checkpoints + backward; 40 KiB 6.55,
// 64 KiB 7.82).
constexpr size_t kBwdLdsBudget = 53 * 1024;
// Filtered steps: two workgroups per CU, each with half the LDS (longer tiles, less per-tile work); the
// kernel's registers allow two workgroups per CU anyway (measured 1.5x faster than 53 KiB at kappa = 20).
constexpr size_t kBwdLdsBudgetFilt = 80 * 1024;

// LDS budget of one backward workgroup; LDBP_BWD_LDS_KIB overrides it (a tuning knob: a smaller
// budget gives more workgroups per CU, a larger one longer tiles and less halo recompute).
static size_t bwd_lds_budget(bool filtered) {
  const char* e = std::getenv("LDBP_BWD_LDS_KIB");
  if (e) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 16 && v <= 160) return static_cast<size_t>(v) * 1024;
  }
  return filtered ? kBwdLdsBudgetFilt : kBwdLdsBudget;
}


struct BwdLayout {
  PassPlan blocks;   // checkpoint blocks (passes of exactly S steps)
  int32_t S;
  int32_t tile_len;
  int64_t ntiles;    // total over the batch
  int32_t ncols;     // sum T + sum(power-filter lengths) + l
  int32_t ntaps;     // sum T
  int32_t neta;      // sum of the power-filter lengths (0 for LDBP)
  size_t off_ckpt, off_g0, off_g1, off_part, off_chunks, total;
  bool stored;       // the caller's checkpoints hold every step's output (ckpt_every = 1): blocks of S steps
                     // read their step outputs instead of recomputing them
};

// Longest block whose stored step outputs the backward kernel loads with its inputs.
constexpr int kMaxStoredSteps = 3;

// Block length of the backward when the caller gives none.  complex64: 2 steps (forward with
// checkpoints + backward on 64 x 65,536, l = 50, 15 taps: S = 1-5 took 2.44, 1.98, 2.11, 2.39, 2.55 ms;
// on 8 x 2^20 x 2, l = 64, 5 taps, with the short-filter kernel variants and the current tile rule:
// S = 2, 3, 4, 5, 6, 8 took 5.22, 5.32, 5.74, 6.31, 9.08, 11.75 ms, and three repeated pairs 5.22-5.26
// against 5.34-5.35 ms for S = 2 and 3); complex128: 3.
static int default_bwd_S(const ModelArgs& m) {
  const int s = m.dtype == LDBP_C64 ? 2 : 3;
  return std::min<int32_t>(m.nstep, s);
}

static int make_bwd_layout(const ModelArgs& m, bool have_ckpt, int32_t ckpt_every, BwdLayout& L) {
  L.S = ckpt_every > 0 ? ckpt_every : default_bwd_S(m);
  // Every step's output given (unfiltered complex64 steps): the backward reads them in blocks of the default length
  // instead of recomputing each step from its checkpoint, trading HBM traffic (S + 3 arrays per block of S
  // steps instead of 3) for the forward FIR and Kerr phase of every step.
  L.stored = have_ckpt && ckpt_every == 1 && !m.filtered() && m.dtype == LDBP_C64 && m.nstep > 1;
  if (L.stored) L.S = std::min(default_bwd_S(m), kMaxStoredSteps);
  int st = make_plan(m, L.S, nullptr, L.blocks);
  if (st) return st;
  // tile length: the largest multiple of 8 whose LDS footprint fits the budget for every block
  size_t budget = bwd_lds_budget(m.filtered());
  int best = 0;
  for (; budget <= kMaxLdsBytes && best == 0; budget += 32 * 1024) {
    for (int Lw = 4096; Lw >= 64; Lw -= 8) {
      bool ok = true;
      for (const auto& pt : L.blocks.passes)
        if (bwd_lds_bytes(m.dtype, m.npol, Lw, pt, m.filtered()) > budget) { ok = false; break; }
      if (ok) { best = Lw; break; }
    }
  }
  if (best == 0)
    return fail(LDBP_EUNSUPPORTED, "checkpoint blocks of %d steps do not fit in LDS for the backward; use fewer",
                L.S);
  // The widest chunked pass, the first recompute step, covers Lw + 4H - 2K_1 samples in rounds of q
  // (outputs per thread x threads).  When its last round would be short, a tile that ends the pass on a
  // whole round does fewer rounds per sample: e.g. 64 x 65,536, l = 50, 15 taps, blocks of 2 steps,
  // q = 1280: 1,256 samples take 2 rounds (1,298 wide), 1,232 one; measured tiles of 1,216 / 1,240 took
  // 1.64 / 1.69 ms per backward, 1,256 2.36 ms.  With one round per pass a tile takes about the same time
  // at any length, so the tiles of a waveform are then made equal (1,216 there); on 8 x 2^20 x 2, 5 taps,
  // blocks of 3 steps, tiles of 632 against 576 took 5.59 against 5.85 ms for forward + backward.
  {
    const int q = bwd_chunk_capacity(m.dtype, m.npol);
    int over = 0;
    for (const auto& pt : L.blocks.passes) over = std::max(over, 4 * pt.halo - 2 * pt.K[0]);
    const int rounds = (best + over + q - 1) / q;
    const int shorter = ((rounds - 1) * q - over) / 8 * 8;
    // rounds per sample: (rounds - 1) / shorter against rounds / best
    if (rounds > 1 && shorter >= 64 && static_cast<int64_t>(rounds - 1) * best < static_cast<int64_t>(rounds) * shorter)
      best = shorter;
    // the same number of tiles per waveform, of equal length (no short last tile)
    const int64_t nt = (m.n + best - 1) / best;
    const int64_t bal = ((m.n + nt - 1) / nt + 7) / 8 * 8;
    if (bal >= 64 && bal < best) best = static_cast<int>(bal);
  }
  // LDBP_BWD_TILE (a tuning knob): an exact tile length, used when it is a multiple of 8 whose LDS
  // footprint fits the largest workgroup allocation
  if (const char* e = std::getenv("LDBP_BWD_TILE")) {
    const long v = std::strtol(e, nullptr, 10);
    bool ok = v >= 64 && v <= 4096 && v % 8 == 0;
    for (const auto& pt : L.blocks.passes)
      if (ok && bwd_lds_bytes(m.dtype, m.npol, static_cast<int>(v), pt, m.filtered()) > kMaxLdsBytes) ok = false;
    if (ok) best = static_cast<int>(v);
  }
  L.tile_len = best;
  L.ntiles = m.nwave * ((m.n + best - 1) / best);
  if (grad_reduce_chunks(L.ntiles) > 65535)
    return fail(LDBP_EUNSUPPORTED, "%lld backward tiles exceed the gradient reduction's grid", (long long)L.ntiles);
  L.ntaps = 0;
  L.neta = 0;
  for (int i = 0; i < m.nstep; ++i) {
    L.ntaps += m.ntap[i];
    if (m.nl_ntap) L.neta += m.nl_ntap[i];
  }
  L.ncols = L.ntaps + L.neta + m.nstep;
  const size_t wave_bytes = static_cast<size_t>(m.nwave) * m.n * m.npol * cx_size(m.dtype);
  const size_t nb = L.blocks.passes.size();
  size_t off = 0;
  L.off_ckpt = off;
  if (!have_ckpt && nb > 1) off += align256((nb - 1) * wave_bytes);
  L.off_g0 = off;
  off += align256(wave_bytes);
  L.off_g1 = off;
  off += align256(wave_bytes);
  L.off_part = off;
  off += align256(static_cast<size_t>(L.ntiles) * L.ncols * sizeof(double) * 2);
  L.off_chunks = off;
  off += align256(static_cast<size_t>(grad_reduce_chunks(L.ntiles)) * L.ncols * sizeof(double) * 2);
  L.total = off;
  return LDBP_OK;
}

}  // namespace ldbp

namespace ldbp {

static int backward_ws_impl(const ModelArgs& m, const void* ckpt, int32_t ckpt_every, size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  int st = check_model(m);
  if (st) return st;
  if (ckpt_every < 0 || ckpt_every > LDBP_MAX_STEPS_PER_PASS)
    return fail(LDBP_EINVAL, "ckpt_every %d outside [0, %d]", ckpt_every, LDBP_MAX_STEPS_PER_PASS);
  if (ckpt && ckpt_every == 0) return fail(LDBP_EINVAL, "ckpt given without ckpt_every");
  BwdLayout L;
  st = make_bwd_layout(m, ckpt != nullptr, ckpt_every, L);
  if (st) return st;
  *bytes = L.total;
  return LDBP_OK;
}

// The backward of LDBP (eta == NULL) and of the generalised ESSM (eta, geta: filters and their gradient).
static int backward_impl(const ModelArgs& m, const void* taps, const void* c, const void* eta, const void* x,
                         const void* ckpt, int32_t ckpt_every, const void* gy, void* gx, void* gtaps, void* gc,
                         void* geta, const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  const int32_t dtype = m.dtype, npol = m.npol;
  const int64_t nwave = m.nwave, n = m.n;
  int st = check_model(m);
  if (st) return st;
  if (plan && (plan->flags & ~(LDBP_PLAN_SYMMETRIC | LDBP_PLAN_ONE_STREAM)))
    return fail(LDBP_EINVAL, "plan flags 0x%x: only LDBP_PLAN_SYMMETRIC and LDBP_PLAN_ONE_STREAM are defined",
                plan->flags);
  const int sym = (plan && (plan->flags & LDBP_PLAN_SYMMETRIC)) ? 1 : 0;
  if (!taps || !c || !x || !gy || !gtaps || !gc)
    return fail(LDBP_EINVAL, "taps, c, x, gy, gtaps and gc must be non-NULL");
  if (m.filtered() && (!eta || !geta)) return fail(LDBP_EINVAL, "eta and geta must be non-NULL");
  if (!aligned16(taps) || !aligned16(x) || !aligned16(gy) || !aligned16(gtaps) || (gx && !aligned16(gx)) ||
      (ckpt && !aligned16(ckpt)))
    return fail(LDBP_EINVAL, "complex arrays must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(c) % real_size(dtype) || reinterpret_cast<uintptr_t>(gc) % real_size(dtype) ||
      (eta && reinterpret_cast<uintptr_t>(eta) % real_size(dtype)) ||
      (geta && reinterpret_cast<uintptr_t>(geta) % real_size(dtype)))
    return fail(LDBP_EINVAL, "c, gc, eta and geta must be aligned to their real type");
  if (ckpt_every < 0 || ckpt_every > LDBP_MAX_STEPS_PER_PASS)
    return fail(LDBP_EINVAL, "ckpt_every %d outside [0, %d]", ckpt_every, LDBP_MAX_STEPS_PER_PASS);
  if (ckpt && ckpt_every == 0) return fail(LDBP_EINVAL, "ckpt given without ckpt_every");
  const size_t wave_bytes = static_cast<size_t>(nwave) * n * npol * cx_size(dtype);
  if (gx && (overlaps(gx, wave_bytes, gy, wave_bytes) || overlaps(gx, wave_bytes, x, wave_bytes)))
    return fail(LDBP_EINVAL, "gx overlaps x or gy");
  BwdLayout L;
  st = make_bwd_layout(m, ckpt != nullptr, ckpt_every, L);
  if (st) return st;
  if (!ws || ws_bytes < L.total)
    return fail(LDBP_EWORKSPACE, "workspace of %zu bytes required, %zu given", L.total, ws ? ws_bytes : 0);
  if (!aligned16(ws)) return fail(LDBP_EINVAL, "ws must be 16-byte aligned");
  if (overlaps(ws, L.total, x, wave_bytes) || overlaps(ws, L.total, gy, wave_bytes) ||
      (gx && overlaps(ws, L.total, gx, wave_bytes)))
    return fail(LDBP_EINVAL, "workspace overlaps an argument");

  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* e = m.filtered() ? eta : nullptr;
  char* wsb = static_cast<char*>(ws);
  void* g0 = wsb + L.off_g0;
  void* g1 = wsb + L.off_g1;
  void* part = wsb + L.off_part;
  const size_t nb = L.blocks.passes.size();
  const char* ck = static_cast<const char*>(ckpt);
  PassPlan bp;  // forward passes that recompute the block inputs 1 .. nb-1 when no checkpoints are given
  if (!ckpt && nb > 1) {
    ck = wsb + L.off_ckpt;
    const int32_t nrun = L.blocks.passes[nb - 1].c0;
    ldbp_plan fp{0, 0, L.blocks.rb, sym ? LDBP_PLAN_SYMMETRIC : 0};
    st = make_block_plan(m, L.S, nrun, &fp, bp);
    if (st) return st;
  }
  const size_t wave_elem_bytes = static_cast<size_t>(n) * npol * cx_size(dtype);
  const int64_t tiles_per_wave = L.ntiles / nwave;
  // launches per half: the forward passes that recompute the block inputs (no checkpoints given), then
  // the blocks from the last to the first
  const size_t nrec = (!ckpt && nb > 1) ? bp.passes.size() : 0;
  st = over_halves(s, nwave, worth_splitting(plan, nb, L.ntiles), nrec + nb,
                   [&](size_t k, int64_t w0, int64_t w1, hipStream_t ss) {
    if (k < nrec)
      return launch_block_pass(m, bp, k, taps, c, x, wsb + L.off_ckpt + (nb - 2) * wave_bytes, wsb + L.off_ckpt,
                               L.S, ss, e, w0, w1);
    const size_t bi = nb - 1 - (k - nrec);
    const size_t off = static_cast<size_t>(w0) * wave_elem_bytes;
    // this range's rows of the partial sums: the tiles of waveforms [w0, w1)
    void* prt = static_cast<double*>(part) + static_cast<size_t>(w0 * tiles_per_wave) * L.ncols * 2;
    // block bi's output gradient: gy for the last block, else the input gradient of block bi + 1
    const char* gcur = static_cast<const char*>(bi + 1 == nb ? gy : (((bi + 1) % 2) ? g1 : g0)) + off;
    const char* xb = (bi == 0 ? static_cast<const char*>(x) : ck + (bi - 1) * wave_bytes) + off;
    const char* ys = nullptr;
    int32_t nstored = 0;
    if (L.stored) {
      // checkpoint j holds the output of step j + 1; the last step's output is not stored (recomputed)
      const int32_t sb = L.blocks.passes[bi].c0;
      xb = (sb == 0 ? static_cast<const char*>(x) : ck + static_cast<size_t>(sb - 1) * wave_bytes) + off;
      ys = ck + static_cast<size_t>(sb) * wave_bytes + off;
      nstored = std::min<int32_t>(L.blocks.passes[bi].nstep, m.nstep - 1 - sb);
    }
    // the block's output is the next block's checkpoint (slot bi): loaded instead of recomputing the
    // block's last step (complex64 steps of one polarisation; the last block's output, y, is not an
    // argument).  Same-box A/B on 64 x 65,536, l = 50, 15 taps: backward 1.415 -> 1.373 ms; with two
    // polarisations the extra array read makes the backward HBM-bound (8 x 2^20 x 2, 5 taps: 4.09 ->
    // 4.33 ms), so they recompute it.
    const char* yout = (!L.stored && dtype == LDBP_C64 && npol == 1 && bi + 1 < nb)
                           ? ck + bi * wave_bytes + off : nullptr;
    char* gin = static_cast<char*>((bi == 0 && gx) ? gx : ((bi % 2) ? g1 : g0)) + off;
    return launch_bwd_block(dtype, npol, xb, gcur, gin, w1 - w0, static_cast<int32_t>(n), L.tile_len,
                            L.blocks.passes[bi], taps, c, prt, L.ncols, L.ntaps + L.neta, sym, ss, e, L.ntaps, ys,
                            static_cast<int64_t>(nwave) * n * npol, nstored, yout);
  });
  if (st) return st;
  return launch_grad_reduce(dtype, part, L.ntiles, L.ncols, L.ntaps, gtaps, gc, s, L.neta, geta, wsb + L.off_chunks);
}

}  // namespace ldbp

extern "C" int ldbp_backward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                            const int32_t* ntap, const void* ckpt, int32_t ckpt_every,
                                            size_t* bytes) {
  return backward_ws_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap}, ckpt, ckpt_every, bytes);
}

extern "C" int ldbp_backward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                             const int32_t* ntap, const void* taps, const void* c, const void* x, const void* ckpt,
                             int32_t ckpt_every, const void* gy, void* gx, void* gtaps, void* gc,
                             const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  return backward_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap}, taps, c, nullptr, x, ckpt, ckpt_every, gy, gx,
                       gtaps, gc, nullptr, plan, ws, ws_bytes, stream);
}

extern "C" int essm_backward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                            const int32_t* ntap, const int32_t* nl_ntap, const void* ckpt,
                                            int32_t ckpt_every, size_t* bytes) {
  if (!nl_ntap) return fail(LDBP_EINVAL, "nl_ntap is NULL");
  return backward_ws_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, ckpt, ckpt_every, bytes);
}

extern "C" int essm_backward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                             const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                             const void* eta, const void* x, const void* ckpt, int32_t ckpt_every, const void* gy,
                             void* gx, void* gtaps, void* gc, void* geta, const ldbp_plan* plan, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!nl_ntap) return fail(LDBP_EINVAL, "nl_ntap is NULL");
  return backward_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, taps, c, eta, x, ckpt, ckpt_every, gy,
                       gx, gtaps, gc, geta, plan, ws, ws_bytes, stream);
}

extern "C" int ldbp_forward_plan_query(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                       const int32_t* ntap, int32_t ckpt_every, const ldbp_plan* plan,
                                       int32_t* npasses, int32_t* tile_len, int32_t* max_steps_per_pass) {
  return plan_query_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap}, ckpt_every, plan, npasses, tile_len,
                         max_steps_per_pass);
}

extern "C" int ldbp_forward_aperiodic_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n,
                                                     int32_t nstep, const int32_t* ntap, const int32_t* nl_ntap,
                                                     int32_t edge, const ldbp_plan* plan, size_t* bytes) {
  return aperiodic_ws_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, edge, plan, bytes);
}

extern "C" int ldbp_forward_aperiodic(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                      const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                                      const void* eta, const void* x, void* y, int32_t edge, const ldbp_plan* plan,
                                      void* ws, size_t ws_bytes, void* stream) {
  return aperiodic_impl(ModelArgs{dtype, npol, nwave, n, nstep, ntap, nl_ntap}, taps, c, eta, x, y, edge, plan, ws,
                        ws_bytes, stream);
}
