/*
 * ldbp.h -- C ABI of the MI355X (gfx950) learned-digital-backpropagation library.
 *
 * Method: Haeger & Pfister, "Physics-Based Deep Learning for Fiber-Optic
 * Communication Systems" (arXiv 2010.14258).  The LDBP model is the
 * parameterised split-step method of eq. (model), Sec. III-B:
 *
 *     f_theta(x) = sigma_l(A^(l) ... sigma_1(A^(1) x)),
 *     A^(i): circular convolution with a centred FIR filter of odd length T_i = 2K_i + 1,
 *            u_m = sum_{k=-K_i}^{K_i} h^(i)_k x_{(m-k) mod n},
 *     sigma_i(u) = u exp(j c_i |u|^2)  (Remark 1; c_i real, sign included).
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) pairs of float (LDBP_C64) or
 *     double (LDBP_C128).  Real parameters (c, step lengths) use the same real type.
 *   - A batch of nwave waveforms of n samples each is stored as [nwave][n][npol]
 *     complex, contiguous.  npol = 2 is dual polarisation (Manakov): both
 *     polarisations share the taps and the phase c_i (|u_x|^2 + |u_y|^2) rotates
 *     both.
 *   - Tap storage: the l filters are packed back to back, filter i occupies
 *     ntap[i] complex values starting at sum_{j<i} ntap[j], index K_i + k
 *     holding h_k (k = -K_i..K_i).  Symmetry is a property of the values only.
 *   - "host" pointers are read during the call only; "device" pointers must be
 *     GPU memory of the current device, 16-byte aligned, and are owned by the
 *     caller.  Inputs and outputs must not overlap unless stated.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *     enqueue work and return without synchronising the host, except where noted.
 *     The multi-pass forward and the backward may run the second half of the batch
 *     on a second stream the library keeps per host thread, device and caller stream
 *     (default priority; at most 16 per thread), forked from `stream` by an event
 *     before its first launch and joined back into it after its last; work enqueued
 *     on `stream` afterwards is ordered after the whole call.  Not while `stream` is
 *     being captured into a graph, and not with LDBP_PLAN_ONE_STREAM.
 *   - Every function returns LDBP_OK (0) or a negative ldbp_status.  Argument
 *     checks run before any GPU work is enqueued; on failure nothing is
 *     enqueued (LDBP_ENONFINITE, the result of a guarded forward, is reported
 *     after its work has run).  ldbp_last_error() returns a thread-local message for the last
 *     failing call.
 *   - The library allocates no device memory inside compute calls; scratch
 *     memory is passed in as a workspace whose size the *_workspace_size
 *     functions report.
 */
#ifndef LDBP_H
#define LDBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ldbp_status {
  LDBP_OK = 0,
  LDBP_EINVAL = -1,       /* invalid argument (size, null pointer, even tap count, alignment, overlap) */
  LDBP_EWORKSPACE = -2,   /* workspace missing or smaller than required */
  LDBP_EUNSUPPORTED = -3, /* valid request the library does not implement (e.g. npol > 2) */
  LDBP_EHIP = -4,         /* a HIP runtime call failed; see ldbp_last_error() */
  LDBP_ENONFINITE = -5    /* guard mode (LDBP_PLAN_GUARD): the forward stored a NaN or an infinity */
};

enum ldbp_dtype { LDBP_C64 = 0, LDBP_C128 = 1 };

#define LDBP_MAX_TAPS 63 /* largest odd filter length per step */
#define LDBP_MAX_NL_TAPS 63 /* largest odd power-filter length per step (generalised ESSM) */
#define LDBP_MAX_STEPS_PER_PASS 64

/* Execution plan of the time-blocked forward.  Zero fields mean "choose".
 *   steps_per_pass      S: number of consecutive FIR+Kerr steps fused in one pass
 *                       (the signal stays in LDS between them; a halo of sum K over
 *                       the S steps is recomputed at each tile edge).
 *   chunks              LDS work size in units of the kernel's chunk (256 threads x
 *                       outputs per thread); the tile length is chunks*chunk - 2*halo.
 *   outputs_per_thread  consecutive outputs each thread computes from one register window
 *                       (c64: 7, 8, 9 for npol 1, 3, 4, 5 for npol 2; c128: 3, 4 / 1, 2).
 *   flags               LDBP_PLAN_SYMMETRIC: the caller guarantees h_{-k} = h_k for every
 *                       filter; the forward then evaluates the folded form
 *                       h_0 x_m + sum_{k>=1} h_k (x_{m-k} + x_{m+k}) (Sec. III-B).
 *                       LDBP_PLAN_ONE_STREAM: every launch goes to `stream` (no split of
 *                       the batch over a second stream).
 *                       LDBP_PLAN_GUARD (ldbp_forward and essm_forward only): non-finite guard.
 *                       The last pass checks every value it stores to y and raises a flag kept
 *                       in 256 bytes of the workspace (ldbp_forward_workspace_size counts
 *                       them); after its launches the call copies the flag to the host,
 *                       which synchronises `stream`, and returns LDBP_ENONFINITE when any
 *                       output is a NaN or an infinity (y is written either way).  The guard
 *                       serves the caller that falls back to plain FFT-DBP when the learned
 *                       model misbehaves; it cannot run inside a graph capture.
 * Zero chunks take the most that still let three workgroups share a compute unit's 160 KiB of
 * LDS; zero steps_per_pass takes steps while twice the pass halo stays within 1/8 of the LDS work
 * size, then spreads the steps evenly over that many passes.
 * Every output is the same sequence of fused multiply-adds whatever the tiling, so results are
 * bit-identical for any steps_per_pass, chunks and outputs_per_thread at fixed
 * LDBP_PLAN_SYMMETRIC, with or without LDBP_PLAN_ONE_STREAM and LDBP_PLAN_GUARD. */
#define LDBP_PLAN_SYMMETRIC 1
#define LDBP_PLAN_ONE_STREAM 2
#define LDBP_PLAN_GUARD 4
typedef struct ldbp_plan {
  int32_t steps_per_pass;
  int32_t chunks;
  int32_t outputs_per_thread;
  int32_t flags;
} ldbp_plan;

/* Library version string and status text. */
const char* ldbp_version(void);
const char* ldbp_status_string(int status);
const char* ldbp_last_error(void);

/* ---------------------------------------------------------------------------
 * LDBP forward: y = f_theta(x) for every waveform of the batch (eq. model, Sec. III-B;
 * nonlinear scaling of Remark 1; Manakov phase for npol = 2).
 *
 *   dtype        LDBP_C64 or LDBP_C128
 *   npol         1 or 2
 *   nwave, n     batch size (>= 1) and samples per waveform (>= 1); circular per waveform
 *   nstep        l >= 1
 *   ntap         host [nstep], odd, 1 <= ntap[i] <= LDBP_MAX_TAPS; any value is
 *                allowed relative to n (wrap-around is part of the definition)
 *   taps         device [sum ntap] complex
 *   c            device [nstep] real
 *   x            device [nwave][n][npol] complex, input
 *   y            device [nwave][n][npol] complex, output; must not overlap x
 *   ckpt         device [ceil(nstep/ckpt_every) - 1][nwave][n][npol] complex or NULL.
 *                When given, the forward runs blocks of ckpt_every steps and
 *                writes the input of block b (b >= 1) to slot b-1; ldbp_backward
 *                recomputes from these instead of storing every step.
 *   ckpt_every   steps per checkpoint block (1..LDBP_MAX_STEPS_PER_PASS) when ckpt != NULL
 *   plan         host, may be NULL (library default); ignored for S when ckpt != NULL
 *   ws           device workspace of at least ldbp_forward_workspace_size() bytes (may be
 *                NULL when that size is 0): the intermediate signal of a multi-pass forward
 *                without checkpoints, and the guard flag with LDBP_PLAN_GUARD
 * -------------------------------------------------------------------------*/
int ldbp_forward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n,
                                int32_t nstep, const int32_t* ntap, const void* ckpt,
                                int32_t ckpt_every, const ldbp_plan* plan, size_t* bytes);

int ldbp_forward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n,
                 int32_t nstep, const int32_t* ntap, const void* taps, const void* c,
                 const void* x, void* y, void* ckpt, int32_t ckpt_every,
                 const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* Execution plan the forward would use: number of passes (kernel launches), the shortest tile
 * length over the passes, and the largest number of fused steps in a pass.  Host only. */
int ldbp_forward_plan_query(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                            const int32_t* ntap, int32_t ckpt_every, const ldbp_plan* plan, int32_t* npasses,
                            int32_t* tile_len, int32_t* max_steps_per_pass);

/* ---------------------------------------------------------------------------
 * Forward without allocation, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation and kernels as ldbp_forward with the same arguments (results bit-identical to
 * ldbp_forward with LDBP_PLAN_ONE_STREAM added to the plan), without ws / ws_bytes: the
 * workspace ldbp_forward_workspace_size would ask for comes from a static device array of
 * LDBP_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the process ends.
 *   - Returns LDBP_EWORKSPACE, before any GPU work, when the call would need more than
 *     LDBP_NOALLOC_SCRATCH_BYTES (a multi-pass forward without checkpoints needs one
 *     intermediate signal, nwave*n*npol complex values, plus 256 bytes with LDBP_PLAN_GUARD).
 *   - Always runs on `stream` alone (LDBP_PLAN_ONE_STREAM is implied).
 *   - Calls no hipMalloc/hipFree; the first call on a device looks up the array's address
 *     on that device (hipGetSymbolAddress) and keeps it.
 *   - Every call on one device shares that device's array: calls that overlap in time on one
 *     device (several streams or host threads) race and must be serialised by the caller.
 * -------------------------------------------------------------------------*/
#define LDBP_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int ldbp_forward_noalloc(int32_t dtype, int32_t npol, int64_t nwave, int64_t n,
                         int32_t nstep, const int32_t* ntap, const void* taps, const void* c,
                         const void* x, void* y, void* ckpt, int32_t ckpt_every,
                         const ldbp_plan* plan, void* stream);

/* ---------------------------------------------------------------------------
 * Generalised enhanced SSM (Sec. III-D, eq. nl_filtered with a filter per step): LDBP whose
 * nonlinear steps filter the power before the phase.  Step i is
 *   u   = h^(i) * x                                        (as in ldbp_forward)
 *   F_j = sum_{k=-kappa_i}^{kappa_i} eta^(i)_k |u_{(j-k) mod n}|^2   (summed over polarisations)
 *   y_j = u_j exp(j c_i F_j)
 * with real filters eta^(i) of odd length nl_ntap[i] = 2 kappa_i + 1.  eta^(i) = (1) is the LDBP
 * step.  Arguments as for ldbp_forward, plus
 *   nl_ntap      host [nstep], odd, 1 <= nl_ntap[i] <= LDBP_MAX_NL_TAPS
 *   eta          device [sum nl_ntap] real (float for LDBP_C64, double for LDBP_C128), filter i at
 *                offset sum_{j<i} nl_ntap[j], index kappa_i + k holding eta_k
 * The halo of a step is K_i + kappa_i; a pass also keeps the power of its tile in LDS.
 * -------------------------------------------------------------------------*/
int essm_forward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                const int32_t* ntap, const int32_t* nl_ntap, const void* ckpt,
                                int32_t ckpt_every, const ldbp_plan* plan, size_t* bytes);

int essm_forward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                 const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                 const void* eta, const void* x, void* y, void* ckpt, int32_t ckpt_every,
                 const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream);

int essm_forward_plan_query(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                            const int32_t* ntap, const int32_t* nl_ntap, int32_t ckpt_every,
                            const ldbp_plan* plan, int32_t* npasses, int32_t* tile_len,
                            int32_t* max_steps_per_pass);

/* ---------------------------------------------------------------------------
 * LDBP backward: gradients of a real loss L through y = f_theta(x).  The paper
 * trains the model with standard tools (Sec. IV-B); this is the chain rule of
 * eq. (model) step by step, with the convention G = dL/dRe + j dL/dIm:
 *   Kerr step  q = Im(G_y conj(y)), dL/dc_i = sum q |u|^2, G_u = (G_y + 2 c_i q y) e^{-j c_i |u|^2}
 *   FIR step   dL/dh_k = sum_m G_u,m conj(x_{m-k}), G_x,p = sum_k conj(h_k) G_u,(p+k)
 * summed over waveforms and polarisations.  The forward is recomputed block by
 * block (ckpt_every steps) from checkpoints, keeping each block's intermediate
 * signals in LDS only; for complex64 steps of one polarisation, every block but
 * the last reads its own output from the next checkpoint instead of recomputing
 * its last step (the same values bit for bit: the forward's outputs do
 * not depend on the tiling).  Sums over samples are formed per tile and reduced in
 * FP64 in a fixed order: results are deterministic.
 *
 *   (dtype .. c)  as for ldbp_forward
 *   x            device [nwave][n][npol] complex: the forward input
 *   ckpt         device checkpoints written by ldbp_forward with the same x, taps, c,
 *                ckpt_every and LDBP_PLAN_SYMMETRIC flag, or NULL: the backward recomputes
 *                them into its workspace.  With
 *                ckpt_every = 1 (every step's output stored; complex64, ldbp_backward only)
 *                the backward reads the stored outputs in blocks of the default length
 *                instead of recomputing each step (more HBM traffic, fewer instructions)
 *   ckpt_every   block length S (1..LDBP_MAX_STEPS_PER_PASS); 0 = library default
 *                (only with ckpt == NULL: 2 steps for complex64, 3 for complex128, or
 *                nstep if smaller).  Long blocks may not fit in LDS
 *                (LDBP_EUNSUPPORTED).
 *   gy           device [nwave][n][npol] complex: dL/dy
 *   gx           device [nwave][n][npol] complex output dL/dx, or NULL when not needed
 *   gtaps        device [sum ntap] complex output, overwritten
 *   gc           device [nstep] real output, overwritten
 *   plan         host, may be NULL; only flags is used.  LDBP_PLAN_SYMMETRIC: the caller
 *                guarantees h_{-k} = h_k; the three FIR products (recompute, adjoint, tap
 *                correlation) are evaluated folded, and gtaps holds the gradient projected on
 *                symmetric filters: entries k and -k both hold (dL/dh_k + dL/dh_{-k}) / 2, the
 *                centre dL/dh_0 (so their sum over a mirrored pair is the gradient of the shared
 *                parameter).  LDBP_PLAN_ONE_STREAM as for the forward.  Other flag bits:
 *                LDBP_EINVAL.
 *   ws           device workspace of ldbp_backward_workspace_size() bytes
 * -------------------------------------------------------------------------*/
int ldbp_backward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                 const int32_t* ntap, const void* ckpt, int32_t ckpt_every, size_t* bytes);

int ldbp_backward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                  const int32_t* ntap, const void* taps, const void* c, const void* x,
                  const void* ckpt, int32_t ckpt_every, const void* gy, void* gx, void* gtaps,
                  void* gc, const ldbp_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Generalised ESSM backward: gradients of a real loss through essm_forward (the chain rule of
 * eq. nl_filtered with a filter per step; the paper trains with standard tools).  For a step with
 * phi = c F, F = eta * P, P = |u|^2 and q = Im(G_y conj(y)) = dL/dphi:
 *   dL/dc = sum_j q_j F_j,  dL/deta_k = c sum_j q_j P_{j-k},  r_m = c sum_k eta_k q_{m+k},
 *   G_u = G_y e^{-j phi} + 2 r u,
 * and the FIR step as in ldbp_backward.  Arguments as for ldbp_backward, plus nl_ntap and eta as for
 * essm_forward and
 *   geta         device [sum nl_ntap] real output, overwritten
 * Sums over samples are reduced in FP64 in a fixed order (deterministic).
 * -------------------------------------------------------------------------*/
int essm_backward_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                 const int32_t* ntap, const int32_t* nl_ntap, const void* ckpt,
                                 int32_t ckpt_every, size_t* bytes);

int essm_backward(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                  const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                  const void* eta, const void* x, const void* ckpt, int32_t ckpt_every, const void* gy,
                  void* gx, void* gtaps, void* gc, void* geta, const ldbp_plan* plan, void* ws,
                  size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Aperiodic (streaming) forward: the model of ldbp_forward (nl_ntap == NULL) or essm_forward applied
 * to a signal that is not periodic.  The circular FIR of Sec. III-B describes one periodic block;
 * continuous data is processed in blocks with overlap-and-save (Sec. III-A, choice of the block
 * length n).  Here every FIR step is a full linear convolution: the signal is zero before its first
 * and after its last input sample at the input and spreads into those margins by K_i per step.  With
 * P = sum_i (K_i + kappa_i) (kappa_i = (nl_ntap[i] - 1) / 2, 0 for LDBP steps) every output depends
 * only on the inputs within P samples of it.
 *   edge   LDBP_EDGE_ZERO: y [nwave][n][npol] holds that model's output at the n input positions.
 *          LDBP_EDGE_VALID: y [nwave][n - 2P][npol] holds the outputs at input positions P .. n-P-1,
 *          the ones that x determines whatever lies outside it: consecutive chunks of a long
 *          stream, each passed with the P stream samples before and after it, give exactly the
 *          stream's outputs (overlap-save).  n <= 2P: LDBP_EINVAL.
 *   (dtype .. c) as for ldbp_forward; nl_ntap, eta as for essm_forward, or NULL for LDBP steps.
 *   x      device [nwave][n][npol] complex input
 *   plan   as for ldbp_forward (steps_per_pass, chunks, outputs_per_thread, flags)
 *   ws     device workspace of ldbp_forward_aperiodic_workspace_size() bytes (may be 0); the
 *          passes run on n + 2P working samples per waveform (LDBP_EDGE_ZERO) or n (VALID)
 * Results are bit-identical to those of ldbp_forward / essm_forward with the same plan on x padded
 * with P zeros at each end (LDBP_EDGE_ZERO) or on x itself (LDBP_EDGE_VALID), at the output positions.
 * -------------------------------------------------------------------------*/
#define LDBP_EDGE_ZERO 1
#define LDBP_EDGE_VALID 2
int ldbp_forward_aperiodic_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                                          const int32_t* ntap, const int32_t* nl_ntap, int32_t edge,
                                          const ldbp_plan* plan, size_t* bytes);

int ldbp_forward_aperiodic(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, int32_t nstep,
                           const int32_t* ntap, const int32_t* nl_ntap, const void* taps, const void* c,
                           const void* eta, const void* x, void* y, int32_t edge, const ldbp_plan* plan,
                           void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched LDBP inference over uneven waveforms (eq. model for each waveform of the batch).
 * Waveform b has wave_len[b] samples, wave_nstep[b] steps with tap counts
 * step_ntap[sum_{j<b} wave_nstep[j] + s], its own taps and Kerr coefficients.  Packed layouts:
 *   x, y   device [sum_b wave_len[b]][npol] complex (waveforms back to back)
 *   taps   device, all steps of all waveforms back to back, each step ntap centred taps
 *   c      device [sum_b wave_nstep[b]] real
 * Every waveform is processed with all its steps fused in one pass (halo = sum of its K), so the
 * whole batch is one kernel launch over independent (waveform, tile) items ordered by decreasing
 * cost.  A waveform whose total halo leaves less than half an LDS chunk of tile even at the largest
 * work size runs in several passes: its steps in consecutive groups, group g in the (g+1)-th launch,
 * the intermediate signal in a buffer the plan holds (its samples x npol complex values).  The plan
 * owns its device tables and that buffer (allocated by ldbp_batch_plan_create, freed by
 * ldbp_batch_plan_destroy); the forward calls allocate nothing.
 * -------------------------------------------------------------------------*/
typedef struct ldbp_batch_plan ldbp_batch_plan;

/* Host tables are copied; plan may be NULL (outputs_per_thread, chunks and flags are used). */
int ldbp_batch_plan_create(int32_t dtype, int32_t npol, int32_t nwave, const int64_t* wave_len,
                           const int32_t* wave_nstep, const int32_t* step_ntap, const ldbp_plan* plan,
                           ldbp_batch_plan** out);
int ldbp_batch_plan_destroy(ldbp_batch_plan* plan);
/* Totals of the batch: samples, sample x steps, taps, steps; work items and LDS work size. */
int ldbp_batch_plan_info(const ldbp_batch_plan* plan, int64_t* total_samples, int64_t* total_sample_steps,
                         int64_t* total_taps, int64_t* total_steps, int32_t* nitems, int32_t* work);
/* One launch on `stream`. */
int ldbp_batch_forward(const ldbp_batch_plan* plan, const void* taps, const void* c, const void* x, void* y,
                       void* stream);
/* The same launch captured once into a hipGraph (re-captured when any pointer changes) and
 * replayed on `stream`.  Not thread-safe for one plan. */
int ldbp_batch_forward_graph(ldbp_batch_plan* plan, const void* taps, const void* c, const void* x, void* y,
                             void* stream);

/* ---------------------------------------------------------------------------
 * Split-step method (Sec. III-A) for the time-discretised NLSE
 *   du/dz = -(alpha/2) u - j (beta2/2) d^2u/dt^2 + j gamma |u|^2 u      (eq. nlse)
 * on the DFT grid of n samples at rate fs (circular waveforms):
 *   linear step   D(z): X_k <- X_k exp(z (j beta2 w_k^2 / 2 - alpha / 2)), w_k = 2 pi f_k
 *   Kerr step     N(z): x <- x exp(j kerr_scale gamma L_eff(z) |x|^2), L_eff(z) = (1 - e^{-alpha z}) / alpha
 *                 (|x|^2 summed over both polarisations for npol = 2; kerr_scale = 8/9 for Manakov)
 * A link has nspan spans of span_len metres, each cut into nstep steps.  The FFT
 * is hand written for lengths n = 2^a 3^b 5^c, 2 <= n <= 2^24: powers of two in registers
 * (with two polarisations n <= 2^22), other lengths above 4096 with mixed-radix passes in LDS
 * (n = N1 N2 with N1 <= 4096 / npol; EUNSUPPORTED when no such split exists).
 * -------------------------------------------------------------------------*/
typedef struct ssm_link {
  double fs;          /* sampling rate [Hz] */
  double alpha;       /* power attenuation [1/m] (>= 0) */
  double beta2;       /* group-velocity dispersion [s^2/m] */
  double gamma;       /* Kerr coefficient [1/(W m)] */
  double span_len;    /* [m] */
  double kerr_scale;  /* 1 for the scalar NLSE, 8/9 for the Manakov equation */
  double ase_var;     /* channel only: per-sample variance of the complex noise each amplifier adds */
  int32_t nspan;      /* >= 1 */
  int32_t nstep;      /* steps per span, >= 1 */
  const double* step_len; /* host [nstep] step lengths in propagation order (sum = span_len), or NULL = uniform */
  int32_t edfa_gain;  /* 1: amplifier after each span restores the power exactly (gain e^{alpha span_len}) */
  int32_t reserved;
} ssm_link;

/* Workspace for ssm_channel / fft_dbp (step program and FP64-generated twiddle tables). */
int ssm_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link,
                       size_t* bytes);

/* Channel simulator (Sec. III-A, Sec. IV-A): for every span, every step applies N(delta_j) then
 * D(delta_j) (power at the start of the step in the Kerr phase), then the amplifier multiplies by
 * e^{alpha span_len / 2} (if edfa_gain) and adds sqrt(ase_var) * noise[span].
 *   x, y    device [nwave][n][npol] complex; y may equal x (in place), no partial overlap
 *   noise   device [nspan][nwave][n][npol] complex with E|w|^2 = 1, required when ase_var > 0, else
 *           ignored (may be NULL).  ldbp_randn fills such a buffer from a counter-based generator.
 * Synchronises the stream once after uploading the step program. */
int ssm_channel(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link,
                const void* x, void* y, const void* noise, void* ws, size_t ws_bytes, void* stream);

/* FFT digital backpropagation: the exact reverse of ssm_channel without noise.  For spans last to
 * first: multiply by e^{-alpha span_len / 2} (if edfa_gain), then for the steps in reverse order
 * D^{-1}(delta_j) followed by N^{-1}(delta_j).  With gamma = 0 this is the frequency-domain linear
 * equaliser.  r, y as x, y of ssm_channel. */
int fft_dbp(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const ssm_link* link, const void* r,
            void* y, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Uneven batches of the split-step method (Sec. III-A; waveforms of different lengths and span
 * counts over one link, e.g. the serving batch of FFT-based DBP): waveform b has wave_len[b]
 * samples (2^a 3^b 5^c, 2 .. 2^24, all with the mixed-radix passes in LDS) and runs the program of
 * ssm_channel (dbp = 0) or fft_dbp (dbp = 1) for wave_nspan[b] spans of `link` (link->nspan is
 * ignored).  Launches are per program step over all waveforms that still have that step.
 *   ssm_batch_plan_create  validates, builds the per-waveform geometry, programs and FP64 twiddle
 *                          tables in device memory the plan owns (allocated here, once; synchronises
 *                          the device).  Host arrays are copied.  The current device is the plan's.
 *   ssm_batch_plan_info    total samples, total sample x linear steps, the largest number of
 *                          linear steps, and the noise slots a channel plan reads (spans of the
 *                          longest link when ase_var > 0, else 0)
 *   ssm_batch_run          x, y device [sum wave_len][npol] complex, waveforms back to back; y may
 *                          equal x.  noise device [noise_slots][sum wave_len][npol] (slot s = span s
 *                          of every waveform), required when noise_slots > 0, else ignored.
 *                          Asynchronous on `stream`; the plan must not be destroyed before it ends.
 * -------------------------------------------------------------------------*/
typedef struct ssm_batch_plan ssm_batch_plan;
int ssm_batch_plan_create(int32_t dtype, int32_t npol, int32_t nwave, const int64_t* wave_len,
                          const int32_t* wave_nspan, const ssm_link* link, int32_t dbp, ssm_batch_plan** out);
int ssm_batch_plan_destroy(ssm_batch_plan* plan);
int ssm_batch_plan_info(const ssm_batch_plan* plan, int64_t* total_samples, int64_t* total_sample_steps,
                        int32_t* max_steps, int32_t* noise_slots);
int ssm_batch_run(const ssm_batch_plan* plan, const void* x, void* y, const void* noise, void* stream);

/* ---------------------------------------------------------------------------
 * Batched FFT (hand written, n = 2^a 3^b 5^c in [2, 2^24]): y_k = sum_t x_t e^{-+2 pi i k t / n},
 * unnormalised, natural order; inverse != 0 selects the + sign.  x, y device [nwave][n][npol];
 * y may equal x.  The DFT of eq. discretized_nlse (Sec. III-A).
 * -------------------------------------------------------------------------*/
int ldbp_fft_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, size_t* bytes);
int ldbp_fft(int32_t dtype, int32_t npol, int64_t nwave, int64_t n, const void* x, void* y, int32_t inverse,
             void* ws, size_t ws_bytes, void* stream);

/* Transmitter (Sec. IV-A): x(t) = sqrt(P) sum_k s_k p(t - k/R_s) with a root-raised-cosine p of
 * roll-off `rolloff`, periodic frames, sampled at rho samples/symbol (rho and nsym of the form 2^a 3^b 5^c):
 * symbol k sits at sample k*rho, the RRC is applied in the frequency domain and the waveform scaled
 * by sqrt(P) rho (mean power P for unit-energy symbols).  Symbols are 16-QAM,
 * s = (2 (i mod 4) - 3 + j (2 (i div 4) - 3)) / sqrt(10) from indices i in 0..15.
 *   sym_idx device int32 [nwave][nsym][npol]; p_watt device double [nwave];
 *   x device [nwave][rho nsym][npol] complex (output). */
int tx_shape_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, size_t* bytes);
int tx_shape(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs, double rolloff,
             const int32_t* sym_idx, const double* p_watt, void* x, void* ws, size_t ws_bytes, void* stream);

/* The same transmitter for symbols given as values (e.g. the i.i.d. circularly-symmetric Gaussian
 * symbols of the paper's simulations, Sec. IV-A and Table I, drawn with ldbp_randn):
 *   sym device [nwave][nsym][npol] complex of the dtype, read only (unit mean energy gives mean
 *   power P); workspace as tx_shape_workspace_size.  Other arguments and errors as tx_shape. */
int tx_shape_symbols(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs,
                     double rolloff, const void* sym, const double* p_watt, void* x, void* ws, size_t ws_bytes,
                     void* stream);

/* Receiver front end (Sec. IV-A): ideal brick-wall low-pass of two-sided bandwidth equal to the new
 * sampling rate and resampling from n_in to n_out samples per frame (DFT bins |f| < f_out / 2 kept,
 * Nyquist bin zeroed, sample values of in-band signals preserved).  y [nwave][n_in][npol] ->
 * r [nwave][n_out][npol]. */
int rx_lpf_decimate_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t n_in, int64_t n_out,
                                   size_t* bytes);
int rx_lpf_decimate(int32_t dtype, int32_t npol, int64_t nwave, int64_t n_in, int64_t n_out, const void* y,
                    void* r, void* ws, size_t ws_bytes, void* stream);

/* Receiver DSP after equalisation and the training loss (Sec. IV-A, IV-B): matched RRC filter and
 * downsampling by rho (the circulant M), division by sqrt(P), genie phase phi = arg(s^H s~),
 * s^ = s~ e^{-j phi}; per frame (waveform, polarisation) MSE ||s^ - s||^2 / nsym.  With gz != NULL
 * also the gradient of the mean MSE over all frames w.r.t. z (convention dL/dRe + j dL/dIm; phi
 * held fixed, which is exact because it minimises the loss).
 *   z device [nwave][rho nsym][npol]; sym device [nwave][nsym][npol] complex (transmitted symbols);
 *   p_watt device double [nwave]; s_hat (nullable) device [nwave][nsym][npol];
 *   mse device double [nwave * npol]; gz (nullable) device like z. */
int rx_mse_workspace_size(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, size_t* bytes);
int rx_mse(int32_t dtype, int32_t npol, int64_t nwave, int64_t nsym, int32_t rho, double rs, double rolloff,
           const void* z, const void* sym, const double* p_watt, void* s_hat, double* mse, void* gz, void* ws,
           size_t ws_bytes, void* stream);

/* 16-QAM symbols (as in tx_shape) from indices: s device [count] complex. */
int qam16_symbols(int32_t dtype, int64_t count, const int32_t* sym_idx, void* s, void* stream);

/* Counter-based random numbers (Philox4x32-10, Salmon et al., SC'11) for the channel noise and the
 * symbols drawn during training.  Number i of a call uses counter (i/2 low, i/2 high, stream_id
 * low, stream_id high) and key seed; each counter yields 4 words.
 *   ldbp_randbits: out device uint32 [nwords], the words in counter order.
 *   ldbp_randn:    out device [count] complex CN(0, 1) (E|w|^2 = 1): words (a, b) map to
 *                  sqrt(-ln u_a) e^{j 2 pi u_b}, u = (word + 1/2) 2^-32. */
int ldbp_randbits(uint32_t* out, int64_t nwords, uint64_t seed, uint64_t stream_id, void* stream);
int ldbp_randn(int32_t dtype, void* out, int64_t count, uint64_t seed, uint64_t stream_id, void* stream);

/* Adam update (Sec. IV-B; Kingma & Ba constants passed in) on `count` real parameters of the
 * dtype's real type, step t >= 1.  mask (nullable, same type and length): pruned parameters have
 * their gradient and value forced to 0 (Sec. IV-C).  mirror (nullable, device int32
 * [count / comps]): element e of a symmetric filter shares its parameter with element mirror[e],
 * the gradient used is g_e + g_mirror[e] (the centre tap has mirror[e] = e and keeps g_e); comps = 2
 * when the parameters are interleaved complex values, else 1. */
int ldbp_adam(int32_t dtype, void* theta, const void* grad, void* m, void* v, const void* mask,
              const int32_t* mirror, int64_t count, int32_t comps, double lr, double b1, double b2, double eps,
              int64_t t, void* stream);

/* Sum of the rows of a [rows][cols] array of the dtype's real type (complex values as interleaved
 * pairs: cols = 2 x complex count): out[c] = sum_r in[r cols + c], accumulated in FP64 in row order
 * (deterministic).  The gradient of a parameter shared by several steps (one filter in every
 * nonlinear step, Sec. III-D; one span's filters tied across spans) is the sum of the gradients of
 * its copies.  in device [rows][cols], out device [cols], not overlapping; rows >= 1. */
int ldbp_sum_rows(int32_t dtype, const void* in, void* out, int64_t rows, int64_t cols, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LDBP_H */
