// Counter-based Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and a Box-Muller complex normal.
//
// Output number i of a call with key `seed` and 64-bit stream id uses counter
// (i/2 mod 2^32, i/2 >> 32, stream mod 2^32, stream >> 32); the four output words of a counter feed
// complex samples 2p (words 0, 1) and 2p + 1 (words 2, 3).  A word pair (a, b) becomes
// u_a = (a + 1/2) 2^-32, u_b = (b + 1/2) 2^-32 and w = sqrt(-ln u_a) e^{j 2 pi u_b}, so E|w|^2 = 1.
#include "common.h"
#include "txrx_kernels.h"

namespace ldbp {

struct Ph4 {
  uint32_t v[4];
};

__device__ __forceinline__ Ph4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Ph4{{c0, c1, c2, c3}};
}

__global__ void philox_bits(uint32_t* __restrict__ out, int64_t nwords, uint64_t seed, uint64_t stream) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (4 * p >= nwords) return;
  const Ph4 w = philox4x32_10(static_cast<uint32_t>(p), static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32),
                              static_cast<uint32_t>(stream), static_cast<uint32_t>(stream >> 32),
                              static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  for (int i = 0; i < 4; ++i)
    if (4 * p + i < nwords) out[4 * p + i] = w.v[i];
}

template <typename R>
__global__ void philox_cnormal(cx_t<R>* __restrict__ out, int64_t count, uint64_t seed, uint64_t stream) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (2 * p >= count) return;
  const Ph4 w = philox4x32_10(static_cast<uint32_t>(p), static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32),
                              static_cast<uint32_t>(stream), static_cast<uint32_t>(stream >> 32),
                              static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  for (int h = 0; h < 2; ++h) {
    if (2 * p + h >= count) break;
    const double ua = (static_cast<double>(w.v[2 * h]) + 0.5) * 2.3283064365386963e-10;
    const double ub = (static_cast<double>(w.v[2 * h + 1]) + 0.5) * 2.3283064365386963e-10;
    const double r = sqrt(-log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    out[2 * p + h] = cx_t<R>{static_cast<R>(r * c), static_cast<R>(r * s)};
  }
}

int randbits_run(uint32_t* out, int64_t nwords, uint64_t seed, uint64_t stream, hipStream_t s) {
  const int64_t pairs = (nwords + 3) / 4;
  hipLaunchKernelGGL(philox_bits, dim3(static_cast<uint32_t>((pairs + 255) / 256)), dim3(256), 0, s, out, nwords,
                     seed, stream);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

int randn_run(int dtype, void* out, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s) {
  const int64_t pairs = (count + 1) / 2;
  const dim3 grid(static_cast<uint32_t>((pairs + 255) / 256));
  if (dtype == LDBP_C64)
    hipLaunchKernelGGL(philox_cnormal<float>, grid, dim3(256), 0, s, static_cast<float2*>(out), count, seed, stream);
  else
    hipLaunchKernelGGL(philox_cnormal<double>, grid, dim3(256), 0, s, static_cast<double2*>(out), count, seed,
                       stream);
  LDBP_HIP_CHECK(hipGetLastError());
  return LDBP_OK;
}

}  // namespace ldbp
