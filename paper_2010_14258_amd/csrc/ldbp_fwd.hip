// LDBP forward: time-blocked fused FIR + Kerr passes (eq. model, Sec. III-B).
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
#include <algorithm>
#include <vector>

#include "common.h"
#include "ldbp_fir.h"
#include "ldbp_kernels.h"

namespace ldbp {

template <typename R, int NPOL, int RB, int THREADS>
__global__ __launch_bounds__(THREADS) void ldbp_fwd_kernel(const cx_t<R>* __restrict__ x, cx_t<R>* __restrict__ y,
                                                           int32_t n, int32_t tile_len, int32_t ntiles,
                                                           int32_t work, const cx_t<R>* __restrict__ taps,
                                                           const R* __restrict__ c, PassTable pt, int32_t sym,
                                                           cx_t<R>* __restrict__ ckpt, int64_t slot_elems) {
  using V = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  V* b0 = reinterpret_cast<V*>(smem);
  V* b1 = b0 + static_cast<size_t>(work + RB) * NPOL;

  const int tile = static_cast<int>(blockIdx.x % static_cast<uint32_t>(ntiles));
  const int64_t wave = blockIdx.x / static_cast<uint32_t>(ntiles);
  const int t0 = tile * tile_len;
  const int Lw = min(tile_len, n - t0);
  const int H = pt.halo;
  const int W0 = Lw + 2 * H;
  const V* xw = x + wave * static_cast<int64_t>(n) * NPOL;
  V* yw = y + wave * static_cast<int64_t>(n) * NPOL;

  load_tile<R, NPOL, THREADS>(xw, b0, n, t0, H, W0, pt.wrap_general);
  __syncthreads();

  int lo = 0;
  for (int s = 0; s < pt.nstep; ++s) {
    const int K = pt.K[s];
    lo += K;
    const R coef = c[pt.c0 + s] * phase_coef_scale<R>();
    fir_kerr_dispatch<R, NPOL, RB, THREADS>(b0, b1, lo, W0 - lo, K, taps + pt.tapoff[s], coef, sym != 0);
    __syncthreads();
    V* t = b0;
    b0 = b1;
    b1 = t;
    if ((pt.ckpt_mask >> s) & 1) {
      // the next step writes the other buffer, so b0 stays intact while it is copied out
      const int64_t slot = (pt.c0 + s + 1) / pt.ckpt_every - 1;
      V* cw = ckpt + slot * slot_elems + wave * static_cast<int64_t>(n) * NPOL;
      for (int j = threadIdx.x; j < Lw; j += THREADS) {
#pragma unroll
        for (int p = 0; p < NPOL; ++p) cw[static_cast<int64_t>(t0 + j) * NPOL + p] = b0[(H + j) * NPOL + p];
      }
    }
  }

  for (int j = threadIdx.x; j < Lw; j += THREADS) {
#pragma unroll
    for (int p = 0; p < NPOL; ++p) yw[static_cast<int64_t>(t0 + j) * NPOL + p] = b0[(H + j) * NPOL + p];
  }
}

// ---------------------------------------------------------------- host side

// Outputs per thread (RB) available for each real type and polarisation count; the chunk of a
// workgroup is 256 * RB samples.  Index 0 is the default.
static constexpr int kThreads = 256;

int fwd_rb_default(int dtype, int npol) {
  if (dtype == LDBP_C64) return npol == 1 ? 7 : 3;
  return npol == 1 ? 3 : 1;
}

bool fwd_rb_supported(int dtype, int npol, int rb) {
  if (dtype == LDBP_C64) return npol == 1 ? (rb == 7 || rb == 8 || rb == 9) : (rb == 3 || rb == 4 || rb == 5);
  return npol == 1 ? (rb == 3 || rb == 4) : (rb == 1 || rb == 2);
}

int fwd_chunk(int dtype, int npol, int rb) {
  (void)dtype;
  (void)npol;
  return kThreads * rb;
}

size_t fwd_lds_bytes(int dtype, int npol, int rb, int chunks) {
  return 2 * static_cast<size_t>(chunks * fwd_chunk(dtype, npol, rb) + rb) * npol * cx_size(dtype);
}

template <typename R, int NPOL, int RB>
static int launch_fwd_pass_t(const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                             const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt,
                             hipStream_t stream) {
  if (pt.ckpt_mask && (!ckpt || pt.ckpt_every < 1)) return fail(LDBP_EINVAL, "checkpoint writes without slots");
  const int work = chunks * RB * kThreads;
  const int tile_len = work - 2 * pt.halo;
  if (tile_len < 1) return fail(LDBP_EINVAL, "pass halo %d too large for work size %d", pt.halo, work);
  const int64_t ntiles = (n + tile_len - 1) / tile_len;
  const int64_t nblocks = ntiles * nwave;
  if (nblocks > 0x7fffffffLL) return fail(LDBP_EUNSUPPORTED, "grid too large (%lld blocks)", (long long)nblocks);
  const size_t lds = 2 * static_cast<size_t>(work + RB) * NPOL * sizeof(cx_t<R>);
  auto kern = ldbp_fwd_kernel<R, NPOL, RB, kThreads>;
  if (lds > 65536) LDBP_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(nblocks)), dim3(kThreads), lds, stream,
                     static_cast<const cx_t<R>*>(x), static_cast<cx_t<R>*>(y), n, tile_len,
                     static_cast<int32_t>(ntiles), work, static_cast<const cx_t<R>*>(taps),
                     static_cast<const R*>(c), pt, sym, static_cast<cx_t<R>*>(ckpt), nwave * n * NPOL);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

int launch_fwd_pass(int dtype, int npol, int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                    const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt, hipStream_t stream) {
#define LDBP_FWD_LAUNCH(R, NP, B)                                                                       \
  if (npol == NP && rb == B)                                                                            \
    return launch_fwd_pass_t<R, NP, B>(x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream);
  if (dtype == LDBP_C64) {
    LDBP_FWD_LAUNCH(float, 1, 7) LDBP_FWD_LAUNCH(float, 1, 8) LDBP_FWD_LAUNCH(float, 1, 9)
    LDBP_FWD_LAUNCH(float, 2, 3) LDBP_FWD_LAUNCH(float, 2, 4) LDBP_FWD_LAUNCH(float, 2, 5)
  } else {
    LDBP_FWD_LAUNCH(double, 1, 3) LDBP_FWD_LAUNCH(double, 1, 4)
    LDBP_FWD_LAUNCH(double, 2, 1) LDBP_FWD_LAUNCH(double, 2, 2)
  }
#undef LDBP_FWD_LAUNCH
  return fail(LDBP_EUNSUPPORTED, "outputs per thread %d not available for this dtype/npol", rb);
}

}  // namespace ldbp
