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
