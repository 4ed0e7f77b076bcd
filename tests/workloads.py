"""Seeded, paper-shaped test inputs built from ``synth`` draws and oracle arithmetic.

Test infrastructure: the waveforms are made on the CPU by the oracle (pulse
shaping, dispersion) from symbols and noise drawn by ``synth``, then handed to
both sides.  The recipe for a received waveform at 2 samples/symbol:
16-QAM symbols -> RRC pulse shaping at launch power P -> a coarse split-step
channel (a few steps per span at the receiver rate, with loss, Kerr effect,
EDFA gain and ASE per span).  It has the bandwidth, power, CD memory and
nonlinear distortion of the received signal of the paper's links without the
cost of a finely resolved simulation at the analog oversampling rate.
"""
from __future__ import annotations

import math

import numpy as np

import synth
from oracle import design as D
from oracle import ssm as S
from oracle import txrx as X
from oracle import units as U

RS = 10.7e9
ALPHA = U.alpha_from_db_per_km(0.2)
BETA2 = U.beta2_from_ps2_per_km(-21.683)
GAMMA = U.gamma_from_per_w_per_km(1.3)


def received_waveforms(seed: int, nwave: int, nsym: int, p_dbm: float, nspan: int = 10, span_km: float = 100.0,
                       rho: int = 2, steps_per_span: int = 2, with_noise: bool = True):
    """Returns (r [nwave, rho*nsym] complex128, symbols [nwave, nsym]).

    Coarse split-step channel at the receiver's sampling rate: ``steps_per_span``
    uniform steps per span (Kerr, dispersion, loss), EDFA gain and ASE per span.
    """
    s = X.qam16(synth.qam16_indices(seed, (nwave, nsym)))
    p = U.dbm_to_watt(p_dbm)
    x = X.tx_shape(s, rho, p, RS)
    fs = rho * RS
    span = span_km * 1e3
    var = U.ase_variance_per_sample(ALPHA, span, 5.0, fs) if with_noise else 0.0
    link = S.Link(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=span, nspan=nspan,
                  step_len=S.uniform_steps(span, steps_per_span), edfa_gain=True, ase_var=var)
    noise = synth.complex_normal(seed + 1, (nspan,) + x.shape) if with_noise else None
    return S.ssm_channel(x, link, noise), s


def ldbp_init(nspan: int, steps_per_span: int, T: int, rho: int = 2, span_km: float = 100.0, kerr_scale: float = 1.0):
    """LS-initialised asymmetric LDBP with log step sizes (Sec. IV-C)."""
    steps = D.log_steps(span_km * 1e3, steps_per_span, ALPHA)
    return D.init_asymmetric(span_km * 1e3, nspan, steps, T, rho * RS, ALPHA, BETA2, GAMMA, kerr_scale=kerr_scale)


def pack_taps(taps):
    return np.concatenate([np.asarray(h, dtype=np.complex128) for h in taps]), [len(h) for h in taps]


def cone_sample(x: np.ndarray, m: int, halo: int) -> np.ndarray:
    """Circular window of x (time axis 0 of a [n] or [n, 2] array) of length 2*halo+1 centred on m."""
    n = x.shape[0]
    idx = (np.arange(-halo, halo + 1) + m) % n
    return x[idx]


def five_smooth_even(v: float) -> int:
    """Nearest even integer whose prime factors are 2, 3 and 5 (FFT-friendly lengths)."""
    best, bd = 2, float("inf")
    lo, hi = int(v * 0.8), int(v * 1.25) + 2
    for m in range(max(2, lo), hi):
        if m % 2:
            continue
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1 and abs(m - v) < bd:
            best, bd = m, abs(m - v)
    return best


def uneven_batch_spec(seed: int, count: int = 256, lo: int = 4096, hi: int = 262144):
    """Lengths (log-uniform, rounded to even 5-smooth), span counts U{1..25}, taps U{3,5,7,9} per waveform."""
    raw = synth.log_uniform_lengths(seed, count, lo, hi)
    lengths = [five_smooth_even(v) for v in raw]
    g = synth.rng(seed, 9)
    nspan = g.integers(1, 26, size=count).tolist()
    taps = g.choice([3, 5, 7, 9], size=count).tolist()
    return lengths, nspan, taps


def unit_peak_gain(h: np.ndarray, grid: int = 4096) -> np.ndarray:
    """Scales a filter so that max_w |sum_k h_k e^{-j k w}| = 1."""
    K = (len(h) - 1) // 2
    w = 2 * np.pi * np.arange(grid) / grid
    H = np.exp(-1j * np.outer(w, np.arange(-K, K + 1))) @ h
    return h / np.max(np.abs(H))


def uneven_models(lengths, nspan, taps, steps_per_span: int = 2, rho: int = 2):
    """Per-waveform LDBP stand-ins: 2 steps per span (log steps), in-band LS taps scaled to unit peak gain.

    Three- to five-tap least-squares filters cascaded over up to 50 steps have out-of-band gains up
    to ~1e5; the amplified out-of-band noise then drives Kerr phases of ~1e5 rad and the model
    becomes chaotic.  Scaling every filter to unit peak gain keeps the cascade non-expansive, as a
    trained serving model would be.
    """
    models = []
    steps = D.log_steps(100e3, steps_per_span, ALPHA)
    one_span = {}
    for n, ns, T in zip(lengths, nspan, taps):
        if T not in one_span:   # every span of the model is the same (same step lengths and positions)
            tp0, c0 = D.init_asymmetric(100e3, 1, steps, T, rho * RS, ALPHA, BETA2, GAMMA, method="inband")
            one_span[T] = ([unit_peak_gain(h) for h in tp0], c0)
        tp, c = one_span[T]
        models.append((list(tp) * ns, np.tile(c, ns)))
    return models


def cd_received(seed: int, n: int, nspan: int, p_dbm: float = 2.0, rho: int = 2):
    """RRC 16-QAM waveform of n samples after the link's chromatic dispersion plus accumulated ASE."""
    nsym = n // rho
    s = X.qam16(synth.qam16_indices(seed, nsym))
    x = X.tx_shape(s, rho, U.dbm_to_watt(p_dbm), RS)
    L = nspan * 100e3
    link = S.Link(fs=rho * RS, alpha=0.0, beta2=BETA2, gamma=0.0, span_len=L, nspan=1, step_len=[L], edfa_gain=False)
    r = S.lin_step(x, L, link)
    var = nspan * U.ase_variance_per_sample(ALPHA, 100e3, 5.0, rho * RS)
    return r + math.sqrt(var) * synth.complex_normal(seed + 7, n)
