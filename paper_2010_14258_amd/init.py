"""Host-side parameter initialisation for LDBP (Sec. IV-C): units, step sizes, taps, Kerr coefficients.

These run once per model on the CPU (a few hundred small vectors) and produce
the device parameters the kernels train and apply.

  * log step sizes: every step of a span carries the same integral of
    exp(-alpha' z), alpha' = 0.4 alpha (the logarithmic heuristic the paper
    adopts with adjusting factor 0.4), so steps are short where the power is high;
  * taps: least-squares fit of the inverse-dispersion response exp(j xi w^2),
    xi = -beta2 delta f_s^2 / 2.  Default ("inband"): the error is weighted 1
    inside the signal band |w| <= pi (1 + rolloff) / rho and sqrt(mu) outside,
    against the same all-pass target, which keeps the out-of-band gain near one
    (the paper fits in band with bounded out-of-band gain); solved from the T x T
    normal equations, whose matrix is Hermitian Toeplitz.  "full": the full-band
    fit, which on an N-point grid is the truncated inverse DFT of the response,
    computed with one FFT;
  * unit filters (h_0 = 1) and random filters (real and imaginary parts i.i.d. N(0, 1), each filter
    divided by the sum of its squared magnitudes), the alternatives the paper compares with the
    least-squares filters (Sec. V-E);
  * Kerr coefficients: c = -kerr_scale gamma L_eff(delta) e^{-alpha z_a} for the
    forward step that starts at span position z_a (unit-gain filters keep the
    signal at launch power, so the span's power profile is carried by c).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def db_per_km_to_alpha(db_per_km: float) -> float:
    return db_per_km * math.log(10.0) / 10.0 / 1e3


def ps2_per_km_to_beta2(v: float) -> float:
    return v * 1e-27


def dbm_to_w(p_dbm: float) -> float:
    return 10.0 ** (p_dbm / 10.0 - 3.0)


def effective_length(z: float, alpha: float) -> float:
    return z if alpha == 0.0 else -math.expm1(-alpha * z) / alpha


def ase_variance(alpha: float, span_len: float, nf_db: float, fs: float, nu: float = 1.946e14,
                 planck: float = 6.626e-34) -> float:
    """Per-sample complex noise variance of one amplifier: PSD (e^{alpha L} - 1) h nu n_sp times fs."""
    g = math.exp(alpha * span_len)
    n_sp = 10.0 ** (nf_db / 10.0) / (2.0 * (1.0 - 1.0 / g))
    return (g - 1.0) * planck * nu * n_sp * fs


def log_step_sizes(span_len: float, nstep: int, alpha: float, factor: float = 0.4) -> List[float]:
    a = factor * alpha
    if nstep == 1 or a == 0.0:
        return [span_len / nstep] * nstep
    total = -math.expm1(-a * span_len)            # integral of a e^{-a z} over the span
    bounds = [0.0]
    for j in range(1, nstep):
        bounds.append(-math.log1p(-total * j / nstep) / a)
    bounds.append(span_len)
    return [bounds[j + 1] - bounds[j] for j in range(nstep)]


def inverse_cd_taps(delta: float, beta2: float, fs: float, ntap: int, grid: int = 4096) -> np.ndarray:
    """Centred taps h_{-K..K} of the full-band least-squares fit to exp(j xi w^2) (truncated inverse DFT)."""
    xi = -beta2 * delta * fs * fs / 2.0
    w = 2.0 * np.pi * np.fft.fftfreq(grid)          # FFT-ordered grid of angular frequencies
    resp = np.exp(1j * xi * w * w)
    h_all = np.fft.ifft(resp)                        # h_all[k mod grid] = (1/N) sum_m resp_m e^{j k w_m}
    K = (ntap - 1) // 2
    return np.array([h_all[k % grid] for k in range(-K, K + 1)])


def inverse_cd_taps_inband(delta: float, beta2: float, fs: float, ntap: int, rho: int = 2, rolloff: float = 0.1,
                           mu: float = 1e-3, grid: int = 4096) -> np.ndarray:
    """Weighted least squares: weight 1 for |w| <= pi (1 + rolloff) / rho, sqrt(mu) outside (grid of N+1 points)."""
    xi = -beta2 * delta * fs * fs / 2.0
    K = (ntap - 1) // 2
    w = 2.0 * np.pi * np.arange(-grid // 2, grid // 2 + 1) / grid
    wt2 = np.where(np.abs(w) <= np.pi * (1.0 + rolloff) / rho, 1.0, mu)   # squared weights
    resp = np.exp(1j * xi * w * w)
    lags = np.arange(-2 * K, 2 * K + 1)
    # normal equations: G[a, b] = sum_i wt2 e^{j (a - b) w_i}, rhs[a] = sum_i wt2 e^{j a w_i} resp_i
    r = np.array([np.sum(wt2 * np.exp(1j * l * w)) for l in lags])
    k = np.arange(-K, K + 1)
    G = r[(k[:, None] - k[None, :]) + 2 * K]
    rhs = np.array([np.sum(wt2 * np.exp(1j * a * w) * resp) for a in k])
    return np.linalg.solve(G, rhs)


def multi_objective_taps(taps: Sequence[np.ndarray], xis: Sequence[float], rho: int = 2, rolloff: float = 0.1,
                         mu: float = 1e-3, max_window: int = 0, sweeps: int = 3, grid: int = 1024,
                         history: list = None) -> List[np.ndarray]:
    """Joint filter design as a multi-objective weighted least-squares problem (Sec. VI-B, eqs.
    objectives and weighted_ls): besides each response F(h_i) ~ e^{j xi_i w^2}, the response of every
    run of neighbouring filters F(h_a * ... * h_b) ~ e^{j (xi_a + ... + xi_b) w^2} (runs of up to
    max_window filters; 0 = all).  With all filters but h_i fixed, the runs containing i give the
    weighted LS problem  min_h sum_runs || (B h) o e_run - d_run ||^2_W  with e_run the product of the
    other filters' responses, d_run the run's target and W the in-band weights of
    inverse_cd_taps_inband; the filters are updated in turn for `sweeps` passes (block coordinate
    descent, so the total objective never increases).  All runs weigh the same.  taps: the starting
    filters (odd lengths, e.g. the individual fits); returns the new filters.  history (a list):
    receives the total objective before the first and after every sweep."""
    M = len(taps)
    L = M if max_window <= 0 else min(max_window, M)
    w = 2.0 * np.pi * np.arange(-grid // 2, grid // 2 + 1) / grid
    wt2 = np.where(np.abs(w) <= np.pi * (1.0 + rolloff) / rho, 1.0, mu)
    Ks = [(len(h) - 1) // 2 for h in taps]
    Bs = [np.exp(-1j * np.outer(w, np.arange(-K, K + 1))) for K in Ks]   # response = B h = sum_k h_k e^{-j k w}
    hs = [np.asarray(h, dtype=np.complex128).copy() for h in taps]
    H = [B @ h for B, h in zip(Bs, hs)]
    ph = [np.exp(1j * x * w * w) for x in xis]

    def total():
        J = 0.0
        for a in range(M):
            prod, tgt = np.ones_like(w, dtype=np.complex128), np.ones_like(w, dtype=np.complex128)
            for b in range(a, min(M, a + L)):
                prod = prod * H[b]
                tgt = tgt * ph[b]
                J += float(np.sum(wt2 * np.abs(prod - tgt) ** 2))
        return J

    if history is not None:
        history.append(total())
    for _ in range(sweeps):
        for i in range(M):
            A = np.zeros((len(hs[i]), len(hs[i])), dtype=np.complex128)
            rhs = np.zeros(len(hs[i]), dtype=np.complex128)
            left, ltgt = np.ones_like(w, dtype=np.complex128), np.ones_like(w, dtype=np.complex128)
            for a in range(i, max(-1, i - L), -1):        # runs start at a <= i ...
                if a < i:
                    left = left * H[a]
                    ltgt = ltgt * ph[a]
                right, rtgt = np.ones_like(w, dtype=np.complex128), np.ones_like(w, dtype=np.complex128)
                for b in range(i, min(M, a + L)):         # ... and end at b >= i
                    if b > i:
                        right = right * H[b]
                        rtgt = rtgt * ph[b]
                    e = left * right
                    d = ltgt * ph[i] * rtgt
                    Be = Bs[i] * e[:, None]
                    A += Be.conj().T @ (wt2[:, None] * Be)
                    rhs += Be.conj().T @ (wt2 * d)
            hs[i] = np.linalg.solve(A, rhs)
            H[i] = Bs[i] @ hs[i]
        if history is not None:
            history.append(total())
    return hs


def ldbp_parameters_symmetric(span_len: float, nspan: int, steps_per_span: int, ntap, fs: float, alpha: float,
                              beta2: float, gamma: float, kerr_scale: float = 1.0, log_steps: bool = True,
                              method: str = "inband", rho: int = 2, rolloff: float = 0.1, mu: float = 1e-3):
    """Symmetric-SSM LDBP (Sec. III-C, IV-C): M = nspan * steps_per_span nonlinear steps and l = M + 1
    linear ones -- the first and last half-steps and, between nonlinear steps, the merged halves of the
    two neighbouring steps -- so the model's last step is linear only (c_l = 0).  Returns (taps, c)."""
    steps = (log_step_sizes(span_len, steps_per_span, alpha) if log_steps
             else [span_len / steps_per_span] * steps_per_span)
    sched = backprop_schedule(span_len, nspan, steps)
    deltas = [d for d, _ in sched]
    merged = ([deltas[0] / 2.0] + [(deltas[i - 1] + deltas[i]) / 2.0 for i in range(1, len(deltas))]
              + [deltas[-1] / 2.0])
    L = len(merged)
    ts = [int(ntap)] * L if np.isscalar(ntap) else [int(t) for t in ntap]
    taps = []
    for i, d in enumerate(merged):
        if method == "inband":
            taps.append(inverse_cd_taps_inband(d, beta2, fs, ts[i], rho, rolloff, mu))
        else:
            taps.append(inverse_cd_taps(d, beta2, fs, ts[i]))
    c = np.zeros(L)
    for i, (d, z0) in enumerate(sched):
        c[i] = -kerr_scale * gamma * effective_length(d, alpha) * math.exp(-alpha * z0)
    return taps, c


def unit_peak_gain(h: np.ndarray, grid: int = 4096) -> np.ndarray:
    """Scales a filter so that its largest gain over all frequencies is one (non-expansive cascade)."""
    K = (len(h) - 1) // 2
    resp = np.fft.fft(np.concatenate([h[K:], np.zeros(grid - len(h), dtype=complex), h[:K]]))
    return h / np.max(np.abs(resp))


def backprop_schedule(span_len: float, nspan: int, steps: Sequence[float]) -> List[Tuple[float, float]]:
    """(delta, z_start) of the forward steps in the order backpropagation undoes them."""
    starts = np.cumsum([0.0] + list(steps))[:-1]
    order = []
    for _ in range(nspan):
        for j in range(len(steps) - 1, -1, -1):
            order.append((float(steps[j]), float(starts[j])))
    return order


def random_filter(T: int, g: np.random.Generator) -> np.ndarray:
    """T taps with real and imaginary parts i.i.d. N(0, 1), divided by sum_j |h_j|^2 (Sec. V-E)."""
    h = g.standard_normal(T) + 1j * g.standard_normal(T)
    return h / np.sum(np.abs(h) ** 2)


def ldbp_parameters(span_len: float, nspan: int, steps_per_span: int, ntap, fs: float, alpha: float, beta2: float,
                    gamma: float, kerr_scale: float = 1.0, log_steps: bool = True, unit_taps: bool = False,
                    method: str = "inband", rho: int = 2, rolloff: float = 0.1, mu: float = 1e-3,
                    random_seed=None, mo_window: int = 0, mo_sweeps: int = 3):
    """Asymmetric-SSM LDBP (l = nspan * steps_per_span): returns (list of tap vectors, c array).

    unit_taps: unit filters; random_seed (int): random filters (see random_filter) instead of the fit;
    method "multiobjective": the in-band fits refined jointly by multi_objective_taps (runs of up to
    mo_window filters, mo_sweeps passes)."""
    steps = (log_step_sizes(span_len, steps_per_span, alpha) if log_steps
             else [span_len / steps_per_span] * steps_per_span)
    sched = backprop_schedule(span_len, nspan, steps)
    L = len(sched)
    ts = [int(ntap)] * L if np.isscalar(ntap) else [int(t) for t in ntap]
    taps, c = [], np.zeros(L)
    for i, (d, z0) in enumerate(sched):
        if random_seed is not None:
            h = random_filter(ts[i], np.random.Generator(np.random.PCG64([int(random_seed), i])))
        elif unit_taps:
            h = np.zeros(ts[i], dtype=np.complex128)
            h[(ts[i] - 1) // 2] = 1.0
        elif method in ("inband", "multiobjective"):
            h = inverse_cd_taps_inband(d, beta2, fs, ts[i], rho, rolloff, mu)
        else:
            h = inverse_cd_taps(d, beta2, fs, ts[i])
        taps.append(h)
        c[i] = -kerr_scale * gamma * effective_length(d, alpha) * math.exp(-alpha * z0)
    if method == "multiobjective" and not unit_taps and random_seed is None:
        xis = [-beta2 * d * fs * fs / 2.0 for d, _ in sched]
        taps = multi_objective_taps(taps, xis, rho, rolloff, mu, mo_window, mo_sweeps)
    return taps, c
