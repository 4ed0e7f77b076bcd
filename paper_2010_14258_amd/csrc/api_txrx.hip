// C ABI of the batched FFT, transmitter / receiver DSP, random numbers and the Adam update.
#include <cmath>

#include "common.h"
#include "ssm_kernels.h"
#include "txrx_kernels.h"

namespace ldbp {

constexpr size_t kTxMaxLds = 160 * 1024;

static int check_fft(int32_t dtype, int32_t npol, int64_t nwave, int64_t n) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype %d invalid", dtype);
  if (npol != 1 && npol != 2) return fail(LDBP_EUNSUPPORTED, "npol %d not supported", npol);
  if (nwave < 1) return fail(LDBP_EINVAL, "nwave < 1");
  if (!smooth5(n) || n < 2 || n > (int64_t(1) << 24))
    return fail(LDBP_EUNSUPPORTED, "length %lld: lengths 2^a 3^b 5^c in [2, 2^24] are supported", (long long)n);
  if (fft_lds_bytes(dtype, nwave, n, npol) > kTxMaxLds)
    return fail(LDBP_EUNSUPPORTED, "length %lld needs more LDS per workgroup than available", (long long)n);
  return LDBP_OK;
}

static int check_ws(void* ws, size_t have, size_t need) {
  if (need && (!ws || have < need)) return fail(LDBP_EWORKSPACE, "workspace of %zu bytes required, %zu given", need, ws ? have : 0);
  if (ws && !aligned16(ws)) return fail(LDBP_EINVAL, "ws must be 16-byte aligned");
  return LDBP_OK;
}

}  // namespace ldbp

using namespace ldbp;

extern "C" int ldbp_fft_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  int st = check_fft(dtype, npol, nwave, n);
  if (st) return st;
  *bytes = fft_ws_bytes(dtype, nwave, n, npol);
  return LDBP_OK;
}

extern "C" int ldbp_fft(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const void* x, void* y,
                        int32_t inverse, void* ws, size_t ws_bytes, void* stream) {
  int st = check_fft(dtype, npol, nwave, n);
  if (st) return st;
  if (!x || !y || !aligned16(x) || !aligned16(y)) return fail(LDBP_EINVAL, "x and y must be non-NULL and 16-byte aligned");
  const size_t wb = static_cast<size_t>(nwave) * n * npol * cx_size(dtype);
  if (x != y && overlaps(x, wb, y, wb)) return fail(LDBP_EINVAL, "x and y partially overlap");
  const size_t need = fft_ws_bytes(dtype, nwave, n, npol);
  if ((st = check_ws(ws, ws_bytes, need))) return st;
  if (overlaps(ws, need, x, wb) || overlaps(ws, need, y, wb)) return fail(LDBP_EINVAL, "workspace overlaps x or y");
  return fft_run(dtype, nwave, n, npol, x, y, inverse ? 1 : 0, ws, static_cast<hipStream_t>(stream));
}

extern "C" int tx_shape_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho,
                                       size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  if (rho < 1 || !smooth5(rho)) return fail(LDBP_EUNSUPPORTED, "rho must be 2^a 3^b 5^c");
  int st = check_fft(dtype, npol, nwave, nsym);
  if (!st) st = check_fft(dtype, npol, nwave, nsym * rho);
  if (st) return st;
  *bytes = tx_ws_bytes(dtype, nwave, nsym, npol, rho);
  return LDBP_OK;
}

extern "C" int tx_shape(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs,
                        double rolloff, const int32_t* sym_idx, const double* p_watt, void* x, void* ws,
                        size_t ws_bytes, void* stream) {
  size_t need;
  int st = tx_shape_workspace_size(dtype, npol, nwave, nsym, rho, &need);
  if (st) return st;
  if (!(rs > 0) || !(rolloff > 0 && rolloff <= 1)) return fail(LDBP_EINVAL, "need rs > 0 and 0 < rolloff <= 1");
  if (!sym_idx || !p_watt || !x || !aligned16(x)) return fail(LDBP_EINVAL, "sym_idx, p_watt and x must be valid");
  if ((st = check_ws(ws, ws_bytes, need))) return st;
  return tx_run(dtype, nwave, nsym, npol, rho, rs, rolloff, sym_idx, p_watt, x, ws, static_cast<hipStream_t>(stream));
}

extern "C" int tx_shape_symbols(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs,
                                double rolloff, const void* sym, const double* p_watt, void* x, void* ws,
                                size_t ws_bytes, void* stream) {
  size_t need;
  int st = tx_shape_workspace_size(dtype, npol, nwave, nsym, rho, &need);
  if (st) return st;
  if (!(rs > 0) || !(rolloff > 0 && rolloff <= 1)) return fail(LDBP_EINVAL, "need rs > 0 and 0 < rolloff <= 1");
  if (!sym || !aligned16(sym) || !p_watt || !x || !aligned16(x))
    return fail(LDBP_EINVAL, "sym, p_watt and x must be valid (sym and x 16-byte aligned)");
  if ((st = check_ws(ws, ws_bytes, need))) return st;
  const size_t sb = static_cast<size_t>(nwave) * nsym * npol * cx_size(dtype);
  if (overlaps(sym, sb, ws, need)) return fail(LDBP_EINVAL, "sym overlaps the workspace");
  return tx_run(dtype, nwave, nsym, npol, rho, rs, rolloff, nullptr, p_watt, x, ws, static_cast<hipStream_t>(stream),
                sym);
}

extern "C" int rx_lpf_decimate_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n_in,
                                              int64_t n_out, size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  int st = check_fft(dtype, npol, nwave, n_in);
  if (!st) st = check_fft(dtype, npol, nwave, n_out);
  if (st) return st;
  if (n_out > n_in) return fail(LDBP_EINVAL, "n_out must not exceed n_in");
  *bytes = lpf_ws_bytes(dtype, nwave, n_in, n_out, npol);
  return LDBP_OK;
}

extern "C" int rx_lpf_decimate(int32_t dtype, int32_t npol, int64_t nwave, int64_t n_in, int64_t n_out,
                               const void* y, void* r, void* ws, size_t ws_bytes, void* stream) {
  size_t need;
  int st = rx_lpf_decimate_workspace_size(dtype, npol, nwave, n_in, n_out, &need);
  if (st) return st;
  if (!y || !r || !aligned16(y) || !aligned16(r)) return fail(LDBP_EINVAL, "y and r must be valid and aligned");
  if ((st = check_ws(ws, ws_bytes, need))) return st;
  return lpf_run(dtype, nwave, n_in, n_out, npol, y, r, ws, static_cast<hipStream_t>(stream));
}

extern "C" int rx_mse_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho,
                                     size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  if (rho < 1 || !smooth5(rho)) return fail(LDBP_EUNSUPPORTED, "rho must be 2^a 3^b 5^c");
  int st = check_fft(dtype, npol, nwave, nsym);
  if (!st) st = check_fft(dtype, npol, nwave, nsym * rho);
  if (st) return st;
  *bytes = rx_ws_bytes(dtype, nwave, nsym, npol, rho);
  return LDBP_OK;
}

extern "C" int rx_mse(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs,
                      double rolloff, const void* z, const void* sym, const double* p_watt, void* s_hat,
                      double* mse, void* gz, void* ws, size_t ws_bytes, void* stream) {
  size_t need;
  int st = rx_mse_workspace_size(dtype, npol, nwave, nsym, rho, &need);
  if (st) return st;
  if (!(rs > 0) || !(rolloff > 0 && rolloff <= 1)) return fail(LDBP_EINVAL, "need rs > 0 and 0 < rolloff <= 1");
  if (!z || !sym || !p_watt || !mse) return fail(LDBP_EINVAL, "z, sym, p_watt and mse must be non-NULL");
  if (!aligned16(z) || !aligned16(sym) || (s_hat && !aligned16(s_hat)) || (gz && !aligned16(gz)))
    return fail(LDBP_EINVAL, "complex arrays must be 16-byte aligned");
  if ((st = check_ws(ws, ws_bytes, need))) return st;
  return rx_run(dtype, nwave, nsym, npol, rho, rs, rolloff, z, sym, p_watt, s_hat, mse, gz, ws,
                static_cast<hipStream_t>(stream));
}

extern "C" int qam16_symbols(int32_t dtype, int64_t count, const int32_t* sym_idx, void* s, void* stream) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype invalid");
  if (count < 0 || !sym_idx || !s || !aligned16(s)) return fail(LDBP_EINVAL, "invalid arguments");
  if (count == 0) return LDBP_OK;
  return qam_run(dtype, count, sym_idx, s, static_cast<hipStream_t>(stream));
}

extern "C" int ldbp_randbits(uint32_t* out, int64_t nwords, uint64_t seed, uint64_t stream_id, void* stream) {
  if (nwords < 0 || (!out && nwords > 0)) return fail(LDBP_EINVAL, "invalid arguments");
  if (nwords == 0) return LDBP_OK;
  return randbits_run(out, nwords, seed, stream_id, static_cast<hipStream_t>(stream));
}

extern "C" int ldbp_randn(int32_t dtype, void* out, int64_t count, uint64_t seed, uint64_t stream_id, void* stream) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype invalid");
  if (count < 0 || (!out && count > 0) || (out && !aligned16(out))) return fail(LDBP_EINVAL, "invalid arguments");
  if (count == 0) return LDBP_OK;
  return randn_run(dtype, out, count, seed, stream_id, static_cast<hipStream_t>(stream));
}

extern "C" int ldbp_adam(int32_t dtype, void* theta, const void* grad, void* m, void* v, const void* mask,
                         const int32_t* mirror, int64_t count, int32_t comps, double lr, double b1, double b2,
                         double eps, int64_t t, void* stream) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype invalid");
  if (!theta || !grad || !m || !v || count < 0 || t < 1 || (comps != 1 && comps != 2))
    return fail(LDBP_EINVAL, "invalid Adam arguments");
  if (mirror && count % comps) return fail(LDBP_EINVAL, "count must be a multiple of comps with a mirror table");
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0)) return fail(LDBP_EINVAL, "bad Adam constants");
  if (count == 0) return LDBP_OK;
  return adam_run(dtype, theta, grad, m, v, mask, mirror, count, comps, lr, b1, b2, eps, t,
                  static_cast<hipStream_t>(stream));
}

extern "C" int ldbp_sum_rows(int32_t dtype, const void* in, void* out, int64_t rows, int64_t cols, void* stream) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype invalid");
  if (rows < 1 || cols < 0) return fail(LDBP_EINVAL, "rows must be >= 1 and cols >= 0");
  if (!in || !out) return fail(LDBP_EINVAL, "in and out must be non-NULL");
  const size_t rb = real_size(dtype);
  if (reinterpret_cast<uintptr_t>(in) % rb || reinterpret_cast<uintptr_t>(out) % rb)
    return fail(LDBP_EINVAL, "in and out must be aligned to their real type");
  if (overlaps(in, static_cast<size_t>(rows) * cols * rb, out, static_cast<size_t>(cols) * rb))
    return fail(LDBP_EINVAL, "out overlaps in");
  if (cols == 0) return LDBP_OK;
  return sum_rows_run(dtype, in, out, rows, cols, static_cast<hipStream_t>(stream));
}
