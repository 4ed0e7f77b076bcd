// LDBP forward: dual-polarisation complex64 instantiations of the time-blocked pass kernel.
#include "ldbp_fwd_impl.h"

namespace ldbp {

#define LDBP_FWD_ARGS x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite

int launch_fwd_pass_c64p2(int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                          const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt,
                          hipStream_t stream, const void* eta, int64_t slot_elems, const EdgeMap* em,
                          int32_t* nonfinite) {
  if (rb == 3) return launch_fwd_pass_t<float, 2, 3>(LDBP_FWD_ARGS);
  if (rb == 4) return launch_fwd_pass_t<float, 2, 4>(LDBP_FWD_ARGS);
  if (rb == 5) return launch_fwd_pass_t<float, 2, 5>(LDBP_FWD_ARGS);
  return fail(LDBP_EUNSUPPORTED, "outputs per thread %d not available for this dtype/npol", rb);
}

#undef LDBP_FWD_ARGS

}  // namespace ldbp
