// C ABI of the split-step channel simulator and FFT-based DBP: validation and step programs.
#include <cmath>
#include <vector>

#include "common.h"
#include "ssm_kernels.h"

namespace ldbp {

constexpr size_t kSsmMaxLds = 160 * 1024;

static double l_eff(double z, double alpha) { return alpha > 0 ? (1.0 - std::exp(-alpha * z)) / alpha : z; }

static int check_link(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* L) {
  if (dtype != LDBP_C64 && dtype != LDBP_C128) return fail(LDBP_EINVAL, "dtype %d invalid", dtype);
  if (npol != 1 && npol != 2) return fail(LDBP_EUNSUPPORTED, "npol %d not supported", npol);
  if (nwave < 1) return fail(LDBP_EINVAL, "nwave < 1");
  if (!smooth5(n) || n < 2 || n > (int64_t(1) << 24))
    return fail(LDBP_EUNSUPPORTED, "n = %lld: the FFT supports lengths 2^a 3^b 5^c in [2, 2^24]", (long long)n);
  if (!L) return fail(LDBP_EINVAL, "link is NULL");
  if (!(L->fs > 0) || !(L->span_len > 0) || !(L->alpha >= 0) || !std::isfinite(L->beta2) ||
      !std::isfinite(L->gamma) || !std::isfinite(L->kerr_scale) || !(L->ase_var >= 0))
    return fail(LDBP_EINVAL, "link parameters must be finite with fs > 0, span_len > 0, alpha >= 0, ase_var >= 0");
  if (L->nspan < 1 || L->nstep < 1) return fail(LDBP_EINVAL, "nspan and nstep must be >= 1");
  if (L->step_len) {
    double sum = 0;
    for (int j = 0; j < L->nstep; ++j) {
      if (!(L->step_len[j] > 0)) return fail(LDBP_EINVAL, "step_len[%d] must be > 0", j);
      sum += L->step_len[j];
    }
    if (std::fabs(sum - L->span_len) > 1e-6 * L->span_len)
      return fail(LDBP_EINVAL, "step lengths sum to %.9g m, span is %.9g m", sum, L->span_len);
  }
  return LDBP_OK;
}

static double step_of(const ssm_link* L, int j) { return L->step_len ? L->step_len[j] : L->span_len / L->nstep; }

// Channel (Sec. III-A, IV-A): per span, for each step N(delta) then D(delta); after the span the
// amplifier restores the power (exp(alpha L_sp / 2)) and adds noise of variance ase_var.
static void channel_program(const ssm_link* L, bool noise, std::vector<double>& z, std::vector<SsmPw>& pw) {
  const int N = L->nstep;
  const int M = L->nspan * N;
  const double G = L->edfa_gain ? std::exp(0.5 * L->alpha * L->span_len) : 1.0;
  const double sigma = std::sqrt(L->ase_var);
  auto kappa = [&](int j) { return L->kerr_scale * L->gamma * l_eff(step_of(L, j), L->alpha); };
  z.resize(M);
  pw.resize(M + 1);
  for (int i = 0; i < M; ++i) z[i] = step_of(L, i % N);
  pw[0] = SsmPw{0.0, 1.0, 0.0, kappa(0), -1};
  for (int i = 1; i <= M; ++i) {
    const int s = (i - 1) / N, j = (i - 1) % N;
    const bool end = (j == N - 1);
    const bool add = end && noise && L->ase_var > 0;
    pw[i] = SsmPw{0.0, end ? G : 1.0, add ? sigma : 0.0, i < M ? kappa(i % N) : 0.0, add ? s : -1};
  }
}

// Backpropagation: spans last to first; undo the amplifier gain, then for the steps in reverse
// order D^{-1}(delta) followed by N^{-1}(delta).
static void dbp_program(const ssm_link* L, std::vector<double>& z, std::vector<SsmPw>& pw) {
  const int N = L->nstep;
  const int M = L->nspan * N;
  const double gu = L->edfa_gain ? std::exp(-0.5 * L->alpha * L->span_len) : 1.0;
  auto kappa = [&](int j) { return L->kerr_scale * L->gamma * l_eff(step_of(L, j), L->alpha); };
  z.resize(M);
  pw.resize(M + 1);
  for (int i = 0; i < M; ++i) z[i] = -step_of(L, N - 1 - (i % N));
  pw[0] = SsmPw{0.0, gu, 0.0, 0.0, -1};
  for (int i = 1; i <= M; ++i) {
    const int j = N - 1 - ((i - 1) % N);
    pw[i] = SsmPw{-kappa(j), (j == 0 && i < M) ? gu : 1.0, 0.0, 0.0, -1};
  }
}

static int prepare(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* L, SsmGeom& g,
                   int32_t& M) {
  int st = check_link(dtype, npol, nwave, n, L);
  if (st) return st;
  g = make_geom(dtype, nwave, n, npol, L->fs, L->alpha, L->beta2);
  if (ssm_lds_bytes(dtype, g) > kSsmMaxLds)
    return fail(LDBP_EUNSUPPORTED, "n = %lld with npol = %d is beyond the FFT sizes supported (npol 2: n <= 2^22; "
                "other lengths: rows and columns of at most 4096 / npol)", (long long)n, npol);
  M = L->nspan * L->nstep;
  return LDBP_OK;
}

static int run(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* L, bool dbp, const void* x,
               void* y, const void* noise, void* ws, size_t ws_bytes, void* stream) {
  SsmGeom g;
  int32_t M;
  int st = prepare(dtype, npol, nwave, n, L, g, M);
  if (st) return st;
  if (!x || !y) return fail(LDBP_EINVAL, "input and output must be non-NULL");
  if (!aligned16(x) || !aligned16(y) || (noise && !aligned16(noise))) return fail(LDBP_EINVAL, "arrays must be 16-byte aligned");
  const size_t wb = static_cast<size_t>(nwave) * n * npol * cx_size(dtype);
  if (x != y && overlaps(x, wb, y, wb)) return fail(LDBP_EINVAL, "input and output partially overlap");
  if (!dbp && L->ase_var > 0 && !noise) return fail(LDBP_EINVAL, "ase_var > 0 needs a noise buffer");
  const size_t need = ssm_workspace_bytes(dtype, g, M);
  if (!ws || ws_bytes < need) return fail(LDBP_EWORKSPACE, "workspace of %zu bytes required, %zu given", need, ws ? ws_bytes : 0);
  if (!aligned16(ws)) return fail(LDBP_EINVAL, "ws must be 16-byte aligned");
  if (overlaps(ws, need, x, wb) || overlaps(ws, need, y, wb)) return fail(LDBP_EINVAL, "workspace overlaps x or y");
  if (noise) {
    const size_t nb = wb * static_cast<size_t>(L->nspan);
    if (overlaps(noise, nb, y, wb) || overlaps(noise, nb, ws, need)) return fail(LDBP_EINVAL, "noise overlaps y or ws");
  }
  std::vector<double> z;
  std::vector<SsmPw> pw;
  if (dbp) dbp_program(L, z, pw);
  else channel_program(L, noise != nullptr, z, pw);
  return ssm_run(dtype, g, x, y, z, pw, dbp ? nullptr : noise, ws, static_cast<hipStream_t>(stream));
}

}  // namespace ldbp

using namespace ldbp;

extern "C" int ssm_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link,
                                  size_t* bytes) {
  if (!bytes) return fail(LDBP_EINVAL, "bytes is NULL");
  SsmGeom g;
  int32_t M;
  int st = prepare(dtype, npol, nwave, n, link, g, M);
  if (st) return st;
  *bytes = ssm_workspace_bytes(dtype, g, M);
  return LDBP_OK;
}

extern "C" int ssm_channel(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link,
                           const void* x, void* y, const void* noise, void* ws, size_t ws_bytes, void* stream) {
  return run(dtype, npol, nwave, n, link, false, x, y, noise, ws, ws_bytes, stream);
}

extern "C" int fft_dbp(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link, const void* r,
                       void* y, void* ws, size_t ws_bytes, void* stream) {
  return run(dtype, npol, nwave, n, link, true, r, y, nullptr, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------- uneven batches

struct ssm_batch_plan {
  void* impl;
};

extern "C" int ssm_batch_plan_create(int32_t dtype, int32_t npol, int32_t nwave, const int64_t* wave_len,
                                     const int32_t* wave_nspan, const ssm_link* link, int32_t dbp,
                                     ssm_batch_plan** out) {
  if (!out) return fail(LDBP_EINVAL, "out is NULL");
  *out = nullptr;
  if (nwave < 1) return fail(LDBP_EINVAL, "nwave < 1");
  if (!wave_len || !wave_nspan) return fail(LDBP_EINVAL, "wave_len and wave_nspan must be non-NULL");
  if (dbp != 0 && dbp != 1) return fail(LDBP_EINVAL, "dbp must be 0 (channel) or 1 (backpropagation)");
  if (!link) return fail(LDBP_EINVAL, "link is NULL");
  ssm_link L = *link;
  std::vector<std::vector<double>> z(nwave);
  std::vector<std::vector<SsmPw>> pw(nwave);
  for (int32_t b = 0; b < nwave; ++b) {
    if (wave_nspan[b] < 1) return fail(LDBP_EINVAL, "wave_nspan[%d] = %d < 1", b, wave_nspan[b]);
    L.nspan = wave_nspan[b];
    const int st = check_link(dtype, npol, 1, wave_len[b], &L);
    if (st) return st;
    if (dbp) dbp_program(&L, z[b], pw[b]);
    else channel_program(&L, L.ase_var > 0, z[b], pw[b]);
  }
  void* impl = nullptr;
  const int st = ssm_batch_build(dtype, npol, nwave, wave_len, z, pw, L.fs, L.alpha, L.beta2, &impl);
  if (st) return st;
  *out = new ssm_batch_plan{impl};
  return LDBP_OK;
}

extern "C" int ssm_batch_plan_destroy(ssm_batch_plan* plan) {
  if (!plan) return LDBP_OK;
  ssm_batch_free(plan->impl);
  delete plan;
  return LDBP_OK;
}

extern "C" int ssm_batch_plan_info(const ssm_batch_plan* plan, int64_t* total_samples, int64_t* total_sample_steps,
                                   int32_t* max_steps, int32_t* noise_slots) {
  if (!plan) return fail(LDBP_EINVAL, "plan is NULL");
  ssm_batch_totals(plan->impl, total_samples, total_sample_steps, max_steps, noise_slots, nullptr, nullptr, nullptr);
  return LDBP_OK;
}

extern "C" int ssm_batch_run(const ssm_batch_plan* plan, const void* x, void* y, const void* noise, void* stream) {
  if (!plan) return fail(LDBP_EINVAL, "plan is NULL");
  int64_t total = 0;
  int32_t slots = 0, npol = 1, dtype = 0, dev = -1;
  ssm_batch_totals(plan->impl, &total, nullptr, nullptr, &slots, &npol, &dtype, &dev);
  if (!x || !y) return fail(LDBP_EINVAL, "x and y must be non-NULL");
  if (!aligned16(x) || !aligned16(y) || (noise && !aligned16(noise)))
    return fail(LDBP_EINVAL, "arrays must be 16-byte aligned");
  const size_t wb = static_cast<size_t>(total) * npol * cx_size(dtype);
  if (x != y && overlaps(x, wb, y, wb)) return fail(LDBP_EINVAL, "x and y partially overlap");
  if (slots > 0 && !noise) return fail(LDBP_EINVAL, "the plan's channel adds amplifier noise: noise is required");
  if (slots > 0 && overlaps(noise, wb * slots, y, wb)) return fail(LDBP_EINVAL, "noise overlaps y");
  int cur = -1;
  LDBP_HIP_CHECK(hipGetDevice(&cur));
  if (cur != dev) return fail(LDBP_EINVAL, "the plan was created on device %d, device %d is current", dev, cur);
  return ssm_batch_exec(plan->impl, x, y, slots > 0 ? noise : nullptr, static_cast<hipStream_t>(stream));
}
