// Adam update with tap masks and the symmetric-tap parameterisation (Sec. IV-B, IV-C).
//
// theta <- theta - lr m^ / (sqrt(v^) + eps), m^ = m / (1 - b1^t), v^ = v / (1 - b2^t), on real
// parameters (the real and imaginary parts of the taps, the Kerr coefficients).  With a mirror
// table the gradient of a tap is taken w.r.t. the symmetric parameter h_k = h_{-k}, i.e.
// g_k + g_{-k} for both entries (the centre tap keeps g_0), so symmetric filters stay symmetric.
// A mask (0/1 per parameter) removes pruned taps: their gradient and value are forced to zero.
#include "common.h"
#include "txrx_kernels.h"

namespace ldbp {

template <typename R>
__global__ void adam_kernel(R* __restrict__ theta, const R* __restrict__ grad, R* __restrict__ m, R* __restrict__ v,
                            const R* __restrict__ mask, const int32_t* __restrict__ mirror, int64_t count,
                            int32_t comps, double lr, double b1, double b2, double eps, double bc1, double bc2) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= count) return;
  double g = grad[e];
  if (mirror) {
    const int64_t el = e / comps, c = e - el * comps;
    const int64_t me = mirror[el];
    if (me != el) g += grad[me * comps + c];
  }
  const double mk = mask ? static_cast<double>(mask[e]) : 1.0;
  g *= mk;
  const double mm = b1 * m[e] + (1.0 - b1) * g;
  const double vv = b2 * v[e] + (1.0 - b2) * g * g;
  m[e] = static_cast<R>(mm);
  v[e] = static_cast<R>(vv);
  const double upd = lr * (mm / bc1) / (sqrt(vv / bc2) + eps);
  theta[e] = static_cast<R>((theta[e] - upd) * mk);
}

int adam_run(int dtype, void* theta, const void* grad, void* m, void* v, const void* mask, const int32_t* mirror,
             int64_t count, int32_t comps, double lr, double b1, double b2, double eps, int64_t t, hipStream_t s) {
  const double bc1 = 1.0 - pow(b1, static_cast<double>(t));
  const double bc2 = 1.0 - pow(b2, static_cast<double>(t));
  const dim3 grid(static_cast<uint32_t>((count + 255) / 256));
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(adam_kernel<float>, grid, dim3(256), 0, s, static_cast<float*>(theta),
                       static_cast<const float*>(grad), static_cast<float*>(m), static_cast<float*>(v),
                       static_cast<const float*>(mask), mirror, count, comps, lr, b1, b2, eps, bc1, bc2);
  else
    hipLaunchKernelGGL(adam_kernel<double>, grid, dim3(256), 0, s, static_cast<double*>(theta),
                       static_cast<const double*>(grad), static_cast<double*>(m), static_cast<double*>(v),
                       static_cast<const double*>(mask), mirror, count, comps, lr, b1, b2, eps, bc1, bc2);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

// out[c] = sum over r of in[r cols + c], accumulated in FP64 in row order (deterministic): the gradient
// of a parameter shared by several steps is the sum of the gradients of its copies.
template <typename R>
__global__ void sum_rows_kernel(const R* __restrict__ in, R* __restrict__ out, int64_t rows, int64_t cols) {
  const int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int64_t r = 0; r < rows; ++r) acc += static_cast<double>(in[r * cols + c]);
  out[c] = static_cast<R>(acc);
}

int sum_rows_run(int dtype, const void* in, void* out, int64_t rows, int64_t cols, hipStream_t s) {
  const dim3 grid(static_cast<uint32_t>((cols + 255) / 256));
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(sum_rows_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<float*>(out), rows, cols);
  else
    hipLaunchKernelGGL(sum_rows_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                       static_cast<double*>(out), rows, cols);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

}  // namespace ldbp
