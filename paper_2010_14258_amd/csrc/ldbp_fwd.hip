// LDBP forward: host side of the time-blocked passes (kernel in ldbp_fwd_impl.h) and the
// single-polarisation complex64 instantiations; the others live in ldbp_fwd_p2.hip and
// ldbp_fwd_c128.hip so that the three compile in parallel.
#include <algorithm>
#include <vector>

#include "ldbp_fwd_impl.h"

namespace ldbp {

// Outputs per thread (RB) available for each real type and polarisation count; the chunk of a
// workgroup is 256 * RB samples.  Index 0 is the default.
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
  return kFwdThreads * rb;
}

size_t fwd_lds_bytes(int dtype, int npol, int rb, int chunks, bool filtered) {
  const size_t w = static_cast<size_t>(chunks * fwd_chunk(dtype, npol, rb) + rb);
  return 2 * w * npol * cx_size(dtype) + (filtered ? w * real_size(dtype) : 0);
}

int launch_fwd_pass(int dtype, int npol, int rb, const void* x, void* y, int64_t nwave, int32_t n, int32_t chunks,
                    const PassTable& pt, const void* taps, const void* c, int sym, void* ckpt, hipStream_t stream,
                    const void* eta, int64_t slot_elems, const EdgeMap* em, int32_t* nonfinite) {
  if (dtype == LDBP_C64 && npol == 1) {
    if (rb == 7) return launch_fwd_pass_t<float, 1, 7>(x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite);
    if (rb == 8) return launch_fwd_pass_t<float, 1, 8>(x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite);
    if (rb == 9) return launch_fwd_pass_t<float, 1, 9>(x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite);
  } else if (dtype == LDBP_C64) {
    return launch_fwd_pass_c64p2(rb, x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite);
  } else {
    return launch_fwd_pass_c128(npol, rb, x, y, nwave, n, chunks, pt, taps, c, sym, ckpt, stream, eta, slot_elems, em, nonfinite);
  }
  return fail(LDBP_EUNSUPPORTED, "outputs per thread %d not available for this dtype/npol", rb);
}

}  // namespace ldbp
