"""Parameter initialisation for LDBP (Sec. IV-C): step sizes, half-step merging,
least-squares filter taps and per-step Kerr coefficients.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Log step sizes.  The paper uses the logarithmic heuristic of its reference
[Zhang2013c, Eq. (2)] with adjusting factor 0.4 but does not print the formula.
Reading: every step carries the same integral of exp(-alpha' z), alpha' = 0.4
alpha, so that short steps sit where the power is high (span start):
    z_j = -ln(1 - (j/N)(1 - e^{-alpha' L_sp})) / alpha',   j = 0..N,
    delta_j = z_j - z_{j-1}  (propagation order).
This reproduces Example 1 (100 km, 2 steps: 29.6 / 70.4 km).

Half-step merging (Sec. IV-C, symmetric SSM): delta'_1 = delta_1/2,
delta'_i = (delta_{i-1} + delta_i)/2, delta'_{M+1} = delta_M/2, with the deltas
listed in the order backpropagation visits them.

Least-squares taps (Sec. IV-C): minimise ||B h - d||^2 with d_i = e^{j xi w_i^2},
xi = -beta2 delta' f_s^2 / 2, w_i = 2 pi i / N for i = -N/2..N/2 and B the
(N+1) x T DFT matrix B_{i,k} = e^{-j k w_i} (centred DTFT of the taps).  The
full-band fit on the N-point grid is exactly the truncated inverse DFT of the
response.  The paper instead fits only within the signal bandwidth and bounds
the out-of-band gain, citing [Sheikh2016] for the details, which the paper does
not give.  Reading: a weighted least-squares fit with weight 1 for
|w| <= pi (1 + rolloff) / rho (the RRC signal band at rho samples/symbol) and
weight sqrt(mu) elsewhere, against the same all-pass target everywhere; the
small out-of-band weight keeps the gain there near one instead of letting the
cascade of filters amplify out-of-band noise.  mu = 1e-3 by default
("inband" method).  Parity of this reading against the cited method: unpinned.

Kerr coefficients: a DBP step that undoes forward step delta starting at span
position z_a uses c = -kerr_scale * gamma * L_eff(delta) * e^{-alpha z_a}: the
LDBP filters have unit gain, so the signal keeps the launch-power level and the
span's power profile is carried by c instead.

Multi-objective design (Sec. VI-B): every run of neighbouring filters adds one
weighted LS objective on its combined response; with all other filters fixed the
objectives of one filter stack into a single weighted LS problem (eq. weighted_ls),
solved for each filter in turn.  The weights lambda_j and the update order are not
given: all runs weigh the same and filters are updated in step order.

Pins (tests/test_oracle_design.py): Example 1 step sizes and merged lengths and
the identical filters h^(2..4); least squares on the N-point grid equals the
truncated inverse DFT (Parseval); symmetric taps for the even response; the
initialised LDBP with T = n taps reproduces FFT-DBP; T_cd arithmetic (Sec. V-B, V-F);
multi-objective design: single-filter runs give the individual in-band fits, the
total objective of eq. objectives never rises over the updates, and the last
updated filter is a stationary point of it (central differences).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from . import units


def log_steps(span_len: float, nstep: int, alpha: float, factor: float = 0.4) -> list[float]:
    """Logarithmic step sizes of one span, propagation order (reading of Sec. IV-C)."""
    a = factor * alpha
    if a == 0.0 or nstep == 1:
        return [span_len / nstep] * nstep
    z = [-math.log(1.0 - (j / nstep) * (1.0 - math.exp(-a * span_len))) / a for j in range(nstep + 1)]
    z[-1] = span_len
    return [z[j + 1] - z[j] for j in range(nstep)]


def merge_half_steps(deltas: Sequence[float]) -> list[float]:
    """Combine adjacent half-steps of the symmetric SSM (Sec. IV-C): M steps -> M+1 lengths."""
    d = list(deltas)
    out = [d[0] / 2.0]
    for i in range(1, len(d)):
        out.append((d[i - 1] + d[i]) / 2.0)
    out.append(d[-1] / 2.0)
    return out


def xi_of(delta: float, beta2: float, fs: float) -> float:
    """xi = -beta2 delta f_s^2 / 2 (Sec. IV-C, Table I)."""
    return -beta2 * delta * fs * fs / 2.0


def ls_taps(xi: float, T: int, N: int = 4096) -> np.ndarray:
    """Least-squares fit of sum_k h_k e^{-j k w} to e^{j xi w^2} on the paper's (N+1)-point grid."""
    assert T % 2 == 1
    K = (T - 1) // 2
    i = np.arange(-N // 2, N // 2 + 1)
    w = 2.0 * np.pi * i / N
    k = np.arange(-K, K + 1)
    B = np.exp(-1j * np.outer(w, k))
    d = np.exp(1j * xi * w * w)
    h, *_ = np.linalg.lstsq(B, d, rcond=None)
    return h


def ls_taps_inband(xi: float, T: int, band_edge: float, mu: float = 1e-3, N: int = 4096) -> np.ndarray:
    """Weighted LS on the paper's grid: weight 1 for |w| <= band_edge, sqrt(mu) outside (reading above)."""
    assert T % 2 == 1
    K = (T - 1) // 2
    i = np.arange(-N // 2, N // 2 + 1)
    w = 2.0 * np.pi * i / N
    k = np.arange(-K, K + 1)
    wt = np.where(np.abs(w) <= band_edge, 1.0, np.sqrt(mu))
    B = np.exp(-1j * np.outer(w, k)) * wt[:, None]
    d = np.exp(1j * xi * w * w) * wt
    h, *_ = np.linalg.lstsq(B, d, rcond=None)
    return h


def truncated_idft_taps(xi: float, T: int, N: int = 4096) -> np.ndarray:
    """h_k = (1/N) sum_m e^{j xi w_m^2} e^{j k w_m}, w_m = 2 pi m / N, m = -N/2..N/2-1, k = -K..K."""
    K = (T - 1) // 2
    m = np.arange(-N // 2, N // 2)
    w = 2.0 * np.pi * m / N
    d = np.exp(1j * xi * w * w)
    k = np.arange(-K, K + 1)
    return (np.exp(1j * np.outer(k, w)) @ d) / N


def dbp_step_plan(span_len: float, nspan: int, steps_per_span: Sequence[float]):
    """Backpropagation order of (delta, z_start) pairs: spans last to first, steps last to first.

    ``steps_per_span`` lists one span's step lengths in propagation order; z_start
    is the position within the span where that forward step begins.
    """
    starts = np.concatenate([[0.0], np.cumsum(steps_per_span)[:-1]])
    plan = []
    for _ in range(nspan):
        for j in reversed(range(len(steps_per_span))):
            plan.append((float(steps_per_span[j]), float(starts[j])))
    return plan


def kerr_coef(delta: float, z_start: float, alpha: float, gamma: float, kerr_scale: float = 1.0) -> float:
    """c = -kerr_scale gamma L_eff(delta) e^{-alpha z_start} (DBP step for a unit-gain model)."""
    return -kerr_scale * gamma * units.l_eff(delta, alpha) * math.exp(-alpha * z_start)


def init_asymmetric(span_len: float, nspan: int, steps_per_span: Sequence[float], T, fs: float,
                    alpha: float, beta2: float, gamma: float, kerr_scale: float = 1.0,
                    method: str = "ls", N: int = 4096, rho: int = 2, rolloff: float = 0.1, mu: float = 1e-3):
    """LDBP based on the asymmetric SSM, l = M (Sec. IV-C): per-step LS taps and Kerr coefficients.

    ``T`` is an int or a per-layer sequence of odd tap counts.  Returns (taps, c).
    """
    plan = dbp_step_plan(span_len, nspan, steps_per_span)
    L = len(plan)
    Ts = [int(T)] * L if np.isscalar(T) else [int(t) for t in T]
    taps, c = [], np.zeros(L)
    for i, (d, z0) in enumerate(plan):
        xi = xi_of(d, beta2, fs)
        if method == "ls":
            taps.append(ls_taps(xi, Ts[i], N))
        elif method == "inband":
            taps.append(ls_taps_inband(xi, Ts[i], np.pi * (1.0 + rolloff) / rho, mu, N))
        elif method == "truncate":
            taps.append(truncated_idft_taps(xi, Ts[i], N))
        elif method == "unit":
            h = np.zeros(Ts[i], dtype=np.complex128)
            h[(Ts[i] - 1) // 2] = 1.0
            taps.append(h)
        else:
            raise ValueError(method)
        c[i] = kerr_coef(d, z0, alpha, gamma, kerr_scale)
    return taps, c


def init_symmetric(span_len: float, nspan: int, steps_per_span: Sequence[float], T, fs: float,
                   alpha: float, beta2: float, gamma: float, kerr_scale: float = 1.0, N: int = 4096):
    """LDBP based on the symmetric SSM, l = M + 1 with a final linear half-step (Sec. III-C, IV-C)."""
    plan = dbp_step_plan(span_len, nspan, steps_per_span)
    deltas = [d for d, _ in plan]
    merged = merge_half_steps(deltas)
    L = len(merged)
    Ts = [int(T)] * L if np.isscalar(T) else [int(t) for t in T]
    taps = [ls_taps(xi_of(dm, beta2, fs), Ts[i], N) for i, dm in enumerate(merged)]
    c = np.zeros(L)
    for i, (d, z0) in enumerate(plan):
        c[i] = kerr_coef(d, z0, alpha, gamma, kerr_scale)
    return taps, c


def multi_objective_ls(taps: Sequence[np.ndarray], xis: Sequence[float], band_edge: float, mu: float = 1e-3,
                       max_window: int = 0, sweeps: int = 3, N: int = 1024) -> list[np.ndarray]:
    """Joint filter design of Sec. VI-B (eqs. objectives and weighted_ls), written out plainly.

    Objectives: for every run a..b of neighbouring filters (length b - a + 1 <= max_window; 0 = all
    lengths) the combined response F(h^(a) * ... * h^(b)) = prod_m (B h^(m)) should be close to
    e^{j (xi_a + ... + xi_b) w^2} on the (N+1)-point grid w_i = 2 pi i / N, i = -N/2..N/2, with the
    in-band weight of ls_taps_inband (squared weight 1 for |w| <= band_edge, mu outside) and all
    lambda_j = 1.  With every filter but h^(i) held at its current value, each run containing i is one
    term || ((B h^(i)) o e_j - d_j) ||^2_W of eq. weighted_ls, e_j the product of the other filters'
    responses in the run and d_j its target.  The terms are stacked into one weighted matrix and solved
    with one least-squares call; filters are updated in step order (i = 1..M) for `sweeps` passes,
    each update using the filters already updated in the same pass.  Returns the new filters."""
    M = len(taps)
    L = M if max_window <= 0 else min(max_window, M)
    i_grid = np.arange(-N // 2, N // 2 + 1)
    w = 2.0 * np.pi * i_grid / N
    sqrt_wt = np.where(np.abs(w) <= band_edge, 1.0, np.sqrt(mu))
    hs = [np.array(h, dtype=np.complex128) for h in taps]

    def dtft_matrix(T):
        K = (T - 1) // 2
        return np.exp(-1j * np.outer(w, np.arange(-K, K + 1)))

    for _ in range(sweeps):
        for i in range(M):
            Bi = dtft_matrix(len(hs[i]))
            blocks, rhs = [], []
            for a in range(M):
                for b in range(a, M):
                    if not (a <= i <= b) or b - a + 1 > L:
                        continue
                    e = np.ones(len(w), dtype=np.complex128)
                    for m in range(a, b + 1):
                        if m != i:
                            e = e * (dtft_matrix(len(hs[m])) @ hs[m])
                    d = np.exp(1j * sum(xis[a:b + 1]) * w * w)
                    blocks.append(sqrt_wt[:, None] * (e[:, None] * Bi))
                    rhs.append(sqrt_wt * d)
            hs[i], *_ = np.linalg.lstsq(np.vstack(blocks), np.concatenate(rhs), rcond=None)
    return hs


def multi_objective_total(taps: Sequence[np.ndarray], xis: Sequence[float], band_edge: float, mu: float = 1e-3,
                          max_window: int = 0, N: int = 1024) -> float:
    """Sum over the objectives of eq. objectives of the weighted squared errors (all lambda_j = 1)."""
    M = len(taps)
    L = M if max_window <= 0 else min(max_window, M)
    w = 2.0 * np.pi * np.arange(-N // 2, N // 2 + 1) / N
    wt = np.where(np.abs(w) <= band_edge, 1.0, mu)
    J = 0.0
    for a in range(M):
        for b in range(a, min(M, a + L)):
            resp = np.ones(len(w), dtype=np.complex128)
            for m in range(a, b + 1):
                K = (len(taps[m]) - 1) // 2
                resp = resp * (np.exp(-1j * np.outer(w, np.arange(-K, K + 1))) @ taps[m])
            J += float(np.sum(wt * np.abs(resp - np.exp(1j * sum(xis[a:b + 1]) * w * w)) ** 2))
    return J
