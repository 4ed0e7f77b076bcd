// Internal interface of the split-step engine (ssm.hip) used by the C ABI (api_ssm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/ldbp.h"

namespace ldbp {

constexpr int64_t kSsmResidentMax = 4096;

// Geometry of one split-step run, passed to the kernels by value.
struct SsmGeom {
  int64_t n, nwave;
  int32_t npol, resident;
  int32_t N1, N2;    // four-step split n = N1 * N2 (resident: N1 = n, N2 = 1)
  int32_t lo_log;    // log2 of the low twiddle table length
  int32_t pad;
  double fs, alpha, beta2;
};

// Host description of a pointwise operation between linear steps.
struct SsmPw {
  double ka, g, sigma, kb;
  int32_t slot;
};

SsmGeom make_geom(int dtype, int64_t nwave, int64_t n, int npol, double fs, double alpha, double beta2);
size_t ssm_workspace_bytes(int dtype, const SsmGeom& g, int32_t M);
size_t ssm_lds_bytes(int dtype, const SsmGeom& g);
int ssm_run(int dtype, const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
            const std::vector<SsmPw>& pw, const void* noise, void* ws, hipStream_t s);

}  // namespace ldbp
