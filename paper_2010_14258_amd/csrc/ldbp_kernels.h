// Internal launch interface between the C ABI (api_ldbp.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ldbp.h"

namespace ldbp {

// Steps fused in one time-blocked pass.  Passed to the kernels by value.
struct PassTable {
  int32_t nstep;         // steps in this pass
  int32_t halo;          // H = sum of K over the pass
  int32_t c0;            // index of the pass's first step in the global step list
  int32_t wrap_general;  // 1 when H >= n, so tile loads need a full modulo
  uint64_t ckpt_mask;    // bit s: after local step s write the state to checkpoint slot (c0+s+1)/ckpt_every - 1
  int32_t ckpt_every;    // checkpoint block length (used with ckpt_mask)
  int32_t reserved;
  int32_t K[LDBP_MAX_STEPS_PER_PASS];       // half-lengths
  int32_t tapoff[LDBP_MAX_STEPS_PER_PASS];  // offsets into the packed taps
  // filtered nonlinear steps (generalised ESSM; used only when a filter array is passed):
  int32_t kap[LDBP_MAX_STEPS_PER_PASS];     // half-lengths of the real power filters
  int32_t etaoff[LDBP_MAX_STEPS_PER_PASS];  // offsets into the packed filters
};

// Pass input and output of an aperiodic forward (ldbp_forward_aperiodic): on the circle of n working
// samples the pass input is x[g - in_off] for 0 <= g - in_off < in_len (zero elsewhere; the
// waveform stride of x is in_len), and sample g of the result is stored to y[g - out_off] for
// 0 <= g - out_off < out_len (waveform stride out_len).
struct EdgeMap {
  int32_t in_off, in_len, out_off, out_len;
};

// Forward pass kernel geometry: rb = outputs per thread, chunk = 256 * rb samples.
int fwd_rb_default(int dtype, int npol);
bool fwd_rb_supported(int dtype, int npol, int rb);
int fwd_chunk(int dtype, int npol, int rb);
// filtered: the pass also holds the power of the signal (a real per sample) for filtered steps.
size_t fwd_lds_bytes(int dtype, int npol, int rb, int chunks, bool filtered = false);

// ckpt: base of the checkpoint slots written inside the pass (pt.ckpt_mask), or NULL when the mask is 0;
// wave w's state for slot j goes to ckpt + j * slot_elems + w * n * npol (slot_elems 0: nwave * n * npol,
// a larger one when the launch covers a sub-range of a batch whose slots hold every waveform).
// eta: packed real filters of the nonlinear steps (pt.kap / pt.etaoff), or NULL for plain Kerr steps.
// em: NULL, or the aperiodic input/output map of this pass (no checkpoint writes with it).
// nonfinite: NULL, or a device int the pass sets to 1 when it stores a NaN or an infinity to y.
int launch_fwd_pass(int dtype, int npol, int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                    const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt, hipStream_t stream,
                    const void* eta = nullptr, int64_t slot_elems = 0, const EdgeMap* em = nullptr,
                    int32_t* nonfinite = nullptr);

// Instantiation groups of launch_fwd_pass (separate translation units).
int launch_fwd_pass_c64p2(int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                          const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt,
                          hipStream_t stream, const void* eta, int64_t slot_elems, const EdgeMap* em,
                          int32_t* nonfinite);
int launch_fwd_pass_c128(int npol, int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                         const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt,
                         hipStream_t stream, const void* eta, int64_t slot_elems, const EdgeMap* em,
                         int32_t* nonfinite);

// Backward (adjoint) block kernel and the deterministic gradient reduction.
// Partial-sum columns: [taps (ntaps)] [power filters (neta), ecol_base = ntaps] [c (l), ccol_base].
// eta: packed power filters of filtered steps (generalised ESSM), or NULL.
size_t bwd_lds_bytes(int dtype, int npol, int Lw, const PassTable& pt, bool filtered = false);
// Samples one round of a backward workgroup's threads covers in the chunked passes (outputs per thread x
// threads).
int bwd_chunk_capacity(int dtype, int npol);
int launch_bwd_block(int dtype, int npol, const void* xb, const void* gout, void* gin, int64_t nwave, int32_t n,
                     int32_t tile_len, const PassTable& pt, const void* taps, const void* c, void* part,
                     int32_t ncols, int32_t ccol_base, int sym, hipStream_t stream, const void* eta = nullptr,
                     int32_t ecol_base = 0, const void* ys = nullptr, int64_t ys_stride = 0, int32_t nstored = 0,
                     const void* yout = nullptr);
// Two fixed-order stages through chunk_sums (grad_reduce_chunks(ntiles) x ncols double2).
int64_t grad_reduce_chunks(int64_t ntiles);
int launch_grad_reduce(int dtype, const void* part, int64_t ntiles, int32_t ncols, int32_t ntaps, void* gtaps,
                       void* gc, hipStream_t stream, int32_t neta, void* geta, void* chunk_sums);

}  // namespace ldbp
