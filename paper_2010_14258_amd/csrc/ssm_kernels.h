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
  int32_t mixed;     // n > 4096 is not a power of two: the mixed-radix LDS passes of ssm_var.hip
  double fs, alpha, beta2;
};

// One waveform of a mixed-radix (ssm_var.hip) run: n = N1 N2, column tiles of C columns, row tiles of
// RW rows (C and RW powers of two), its program (M linear steps: lengths z[prog ..], pointwise
// operations ops[prog_op .. prog_op + M]) and its twiddle tables (offsets into the table buffer:
// W_N1^k, W_N2^k, W_n^k for k < 2^lo_log, W_n^(k 2^lo_log)).
struct VarWave {
  int64_t off;  // first complex value of the waveform (sample x npol)
  int64_t n;
  int32_t N1, N2, C, RW, ctiles, rtiles, lo_log, M, prog, prog_op;
  int64_t tw1, tw2, tlo, thi;
  uint64_t plan1, plan2;  // radix plans of the N1- and N2-point transforms (fft_radix_plan)
};
struct VarItem {
  int32_t wave, tile;
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

// mixed-radix lengths and uneven batches (ssm_var.hip)
bool smooth5(int64_t n);
int var_geometry(int dtype, int npol, int64_t n, VarWave& w, size_t* lds_bytes);
size_t ssm_var_workspace_bytes(int dtype, int npol, int64_t n);
size_t ssm_var_lds_bytes(int dtype, int npol, int64_t n);
int ssm_run_var(int dtype, const SsmGeom& g, const void* x, void* y, const std::vector<double>& lin_z,
                const std::vector<SsmPw>& pw, const void* noise, void* ws, hipStream_t s);
int ssm_batch_build(int dtype, int npol, int64_t nwave, const int64_t* len, const std::vector<std::vector<double>>& z,
                    const std::vector<std::vector<SsmPw>>& pw, double fs, double alpha, double beta2, void** out);
void ssm_batch_free(void* plan);
void ssm_batch_totals(const void* plan, int64_t* samples, int64_t* sample_steps, int32_t* max_steps,
                      int32_t* slots, int32_t* npol, int32_t* dtype, int32_t* dev);
int ssm_batch_exec(const void* plan, const void* x, void* y, const void* noise, hipStream_t s);

}  // namespace ldbp
