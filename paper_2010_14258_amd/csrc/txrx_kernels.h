// Internal interface of the transmitter / receiver, random-number and optimiser kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ldbp.h"

namespace ldbp {

size_t fft_ws_bytes(int dtype, int64_t nwave, int64_t n, int npol);
size_t fft_lds_bytes(int dtype, int64_t nwave, int64_t n, int npol);
int fft_run(int dtype, int64_t nwave, int64_t n, int npol, const void* x, void* y, int inverse, void* ws,
            hipStream_t s);

size_t tx_ws_bytes(int dtype, int64_t nwave, int64_t nsym, int npol, int rho);
// idx: 16-QAM indices, or NULL with sym: the complex symbols themselves.
int tx_run(int dtype, int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const int32_t* idx,
           const double* p, void* x, void* ws, hipStream_t s, const void* sym = nullptr);
size_t lpf_ws_bytes(int dtype, int64_t nwave, int64_t nin, int64_t nout, int npol);
int lpf_run(int dtype, int64_t nwave, int64_t nin, int64_t nout, int npol, const void* y, void* r, void* ws,
            hipStream_t s);
size_t rx_ws_bytes(int dtype, int64_t nwave, int64_t nsym, int npol, int rho);
int rx_run(int dtype, int64_t nwave, int64_t nsym, int npol, int rho, double rs, double beta, const void* z,
           const void* sym, const double* p, void* shat, double* mse, void* gz, void* ws, hipStream_t s);
int qam_run(int dtype, int64_t count, const int32_t* idx, void* s, hipStream_t st);

int randbits_run(uint32_t* out, int64_t nwords, uint64_t seed, uint64_t stream, hipStream_t s);
int randn_run(int dtype, void* out, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s);

int adam_run(int dtype, void* theta, const void* grad, void* m, void* v, const void* mask, const int32_t* mirror,
             int64_t count, int32_t comps, double lr, double b1, double b2, double eps, int64_t t, hipStream_t s);
int sum_rows_run(int dtype, const void* in, void* out, int64_t rows, int64_t cols, hipStream_t s);

}  // namespace ldbp
