// LDBP forward kernel (included by the files that instantiate it): time-blocked fused FIR + Kerr
// passes (eq. model, Sec. III-B).
//
// One pass applies S consecutive steps u = h * x (circular, centred, T = 2K+1
// taps), y = u exp(j c |u|^2) to a tile of L output samples.  The workgroup
// loads the tile plus a halo of H = sum K over the S steps (wrapping around the
// circular waveform), keeps the signal in LDS between steps (ping-pong buffers),
// and writes only the L samples whose dependency cone was fully loaded.  After
// step s the valid region has shrunk by K_s on each side.  Each thread
// produces RB consecutive outputs from a register window of RB + 2K inputs.
// A pass may span several checkpoint blocks: at an inner block boundary the tile's own L
// samples (valid after every step of the pass) are also written to that block's checkpoint slot.
#pragma once

#include "common.h"
#include "ldbp_fir.h"
#include "ldbp_kernels.h"

namespace ldbp {

constexpr int kFwdThreads = 256;

// One sample to global memory with a non-temporal hint: checkpoints are read back only by the backward,
// long after the pass, so their writes need not stay in the caches.
template <typename R, int NPOL>
__device__ __forceinline__ void store_sample_nt(cx_t<R>* __restrict__ dst, const cx_t<R> (&v)[NPOL]) {
  using vec2 = R __attribute__((ext_vector_type(2)));
  using vec4 = R __attribute__((ext_vector_type(4)));
  if constexpr (NPOL == 2 && sizeof(R) == 4) {
    __builtin_nontemporal_store(vec4{v[0].x, v[0].y, v[1].x, v[1].y}, reinterpret_cast<vec4*>(dst));
  } else {
#pragma unroll
    for (int p = 0; p < NPOL; ++p) __builtin_nontemporal_store(vec2{v[p].x, v[p].y}, reinterpret_cast<vec2*>(dst + p));
  }
}


// FILT: the steps are filtered nonlinear steps (eta != NULL); CKPT: the pass writes inner checkpoints;
// EDGE: the pass input and output follow an EdgeMap (aperiodic forward: zero margins, cropped output).
// Separate instantiations keep the plain LDBP kernel's registers (and occupancy) unchanged.
template <typename R, int NPOL, int RB, int THREADS, bool FILT, bool CKPT, bool EDGE = false>
__global__ __launch_bounds__(THREADS) void ldbp_fwd_kernel(const cx_t<R>* __restrict__ x, cx_t<R>* __restrict__ y,
                                                           int32_t n, int32_t tile_len, int32_t ntiles,
                                                           int32_t work, const cx_t<R>* __restrict__ taps,
                                                           const R* __restrict__ c, PassTable pt, int32_t sym,
                                                           cx_t<R>* __restrict__ ckpt, int64_t slot_elems,
                                                           const R* __restrict__ eta, EdgeMap em,
                                                           int32_t* __restrict__ nonfinite) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  V* b0 = reinterpret_cast<V*>(smem);
  V* b1 = b0 + static_cast<size_t>(work + RB) * NPOL;
  R* pwb = reinterpret_cast<R*>(b1 + static_cast<size_t>(work + RB) * NPOL);  // filtered steps only

  const int tile = static_cast<int>(blockIdx.x % static_cast<uint32_t>(ntiles));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(ntiles);
  const int t0 = tile * tile_len;
  const int Lw = min(tile_len, n - t0);
  const int H = pt.halo;
  const int W0 = Lw + 2 * H;
  const V* xw = x + wave * static_cast<int64_t>(EDGE ? em.in_len : n) * NPOL;
  V* yw = y + wave * static_cast<int64_t>(EDGE ? em.out_len : n) * NPOL;
  // a tile whose samples are all cropped from the output has nothing to do
  if (EDGE && (t0 + Lw <= em.out_off || t0 >= em.out_off + em.out_len)) return;

  if constexpr (EDGE) load_tile_edge<R, NPOL, THREADS>(xw, b0, n, t0, H, W0, pt.wrap_general, em.in_off, em.in_len);
  else load_tile<R, NPOL, THREADS>(xw, b0, n, t0, H, W0, pt.wrap_general);
  __syncthreads();

  int lo = 0;
  for (int s = 0; s < pt.nstep; ++s) {
    const int K = pt.K[s];
    lo += K;
    const R coef = c[pt.c0 + s] * phase_coef_scale<R>();
    if constexpr (FILT) {
      // filtered step: linear part and power, then the phase from the filtered power (the valid
      // region shrinks by K, then by kappa)
      const int kap = pt.kap[s];
      fir_lin_dispatch<R, NPOL, RB, THREADS>(b0, b1, pwb, lo, W0 - lo, K, taps + pt.tapoff[s], sym != 0);
      __syncthreads();
      lo += kap;
      nl_filter_dispatch<R, NPOL, RB, THREADS>(b1, pwb, lo, W0 - lo, kap, eta + pt.etaoff[s], coef);
    } else {
      fir_kerr_dispatch<R, NPOL, RB, THREADS>(b0, b1, lo, W0 - lo, K, taps + pt.tapoff[s], coef, sym != 0);
    }
    __syncthreads();
    V* t = b0;
    b0 = b1;
    b1 = t;
    if (CKPT && ((pt.ckpt_mask >> s) & 1)) {
      // the next step writes the other buffer, so b0 stays intact while it is copied out
      const int64_t slot = (pt.c0 + s + 1) / pt.ckpt_every - 1;
      V* cw = ckpt + slot * slot_elems + wave * static_cast<int64_t>(n) * NPOL;
      for (int j = threadIdx.x; j < Lw; j += THREADS) {
        V v[NPOL];
        load_sample<R, NPOL>(b0 + (H + j) * NPOL, v);
        store_sample_nt<R, NPOL>(cw + static_cast<int64_t>(t0 + j) * NPOL, v);
      }
    }
  }

  bool bad = false;
  for (int j = threadIdx.x; j < Lw; j += THREADS) {
    int o = t0 + j;
    if constexpr (EDGE) {
      o -= em.out_off;
      if (o < 0 || o >= em.out_len) continue;
    }
    V v[NPOL];
    load_sample<R, NPOL>(b0 + (H + j) * NPOL, v);
    // a checkpointing pass writes the next block's checkpoint (or y after the last step)
    if constexpr (CKPT) store_sample_nt<R, NPOL>(yw + static_cast<int64_t>(o) * NPOL, v);
    else store_sample<R, NPOL>(yw + static_cast<int64_t>(o) * NPOL, v);
    if (nonfinite) {
#pragma unroll
      for (int p = 0; p < NPOL; ++p) bad |= !(__builtin_isfinite(v[p].x) && __builtin_isfinite(v[p].y));
    }
  }
  // guard mode: any lane that stored a NaN or an infinity raises the flag (a plain per-lane global
  // store of 1; concurrent writers all write the same value)
  if (bad) *nonfinite = 1;
}

template <typename R, int NPOL, int RB>
inline int launch_fwd_pass_t(const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                             const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt,
                             hipStream_t stream, const void* eta, int64_t slot_elems, const EdgeMap* em,
                             int32_t* nonfinite) {
  if (pt.ckpt_mask && (!ckpt || pt.ckpt_every < 1)) return fail(LDBP_EINVAL, "checkpoint writes without slots");
  if (em && pt.ckpt_mask) return fail(LDBP_EINVAL, "an aperiodic pass writes no checkpoints");
  const int work = chunks * RB * kFwdThreads;
  const int tile_len = work - 2 * pt.halo;
  if (tile_len < 1) return fail(LDBP_EINVAL, "pass halo %d too large for work size %d", pt.halo, work);
  const int64_t ntiles = (n + tile_len - 1) / tile_len;
  const int64_t nblocks = ntiles * nwave;
  if (nblocks > 0x7fffffffLL) return fail(LDBP_EUNSUPPORTED, "grid too large (%lld blocks)", (long long)nblocks);
  const size_t lds = 2 * static_cast<size_t>(work + RB) * NPOL * sizeof(cx_t<R>) +
                     (eta ? static_cast<size_t>(work + RB) * sizeof(R) : 0);
  auto kern = em ? (eta ? ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, true, false, true>
                        : ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, false, false, true>)
           : eta ? (pt.ckpt_mask ? ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, true, true>
                                 : ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, true, false>)
                 : (pt.ckpt_mask ? ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, false, true>
                                 : ldbp_fwd_kernel<R, NPOL, RB, kFwdThreads, false, false>);
  if (lds > 65536) LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(nblocks)), dim3(kFwdThreads), lds, stream,
                     static_cast<const cx_t<R>*>(x), static_cast<cx_t<R>*>(y), n, tile_len,
                     static_cast<int32_t>(ntiles), work, static_cast<const cx_t<R>*>(taps),
                     static_cast<const R*>(c), pt, sym, static_cast<cx_t<R>*>(ckpt),
                     slot_elems > 0 ? slot_elems : nwave * n * NPOL,
                     static_cast<const R*>(eta), em ? *em : EdgeMap{0, n, 0, n}, nonfinite);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

}  // namespace ldbp
