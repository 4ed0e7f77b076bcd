"""Transmitter, receiver DSP, MSE and effective SNR (Sec. IV-A, IV-B).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Transmitter (Sec. IV-A): x(t) = sqrt(P) sum_k s_k p(t - k/R_s), p a root-raised-
cosine (RRC) pulse with 10% roll-off, periodic symbol frames.  Discretised at
rho_a samples/symbol: symbol k is placed at sample k*rho_a (zero insertion), the
RRC is applied in the frequency domain (circular, matching the periodic frame),
and the result is scaled by sqrt(P) * rho_a so that the mean power is P for unit-
energy symbols.  The workloads here use 16-QAM, s = (a + j b)/sqrt(10) with
a, b in {-3, -1, 1, 3}.

Receiver (Sec. IV-A): an ideal brick-wall low-pass of two-sided bandwidth equal to
the new sampling rate (the text's "2 f_s" would alias; Table I gives f_s), then
sampling at rho_d samples/symbol -- done by copying DFT bins with |f| < f_s/2
(Nyquist bin zeroed) and scaling by n_out/n_in so sample values are preserved.
After equalisation: the RRC matched filter, downsampling by rho_d (the circulant
M of Sec. IV-A), division by sqrt(P), and the genie phase correction
phi = arg(s^H s~), s^ = s~ e^{-j phi}.

Loss and figure of merit (Sec. IV-B): MSE = ||s^ - s||^2 / N_sym; the effective
SNR is read as N_sym / E||S^ - S||^2 (the printed expectation of an inverse is
taken as the inverse of the expected error, the only reading under which
minimising the MSE maximises the SNR), pooled over frames, for E|S|^2 = 1.

Arrays: the time axis is ``axis`` (default -1); leading axes are frames.

Pins (tests/test_oracle_txrx.py): back-to-back TX -> LPF/decimate -> MF returns
the symbols exactly; white noise of variance v on the symbols gives SNR -> 1/v;
the RRC satisfies the Nyquist criterion (folded |H|^2 sums to one); the
gradient of the loss w.r.t. the equaliser output against finite differences.
"""
from __future__ import annotations

import numpy as np


def qam16(idx: np.ndarray) -> np.ndarray:
    """16-QAM symbols of unit mean energy from indices 0..15."""
    idx = np.asarray(idx)
    a = 2.0 * (idx % 4) - 3.0
    b = 2.0 * (idx // 4) - 3.0
    return (a + 1j * b) / np.sqrt(10.0)


def rrc_response(n: int, fs: float, rs: float, rolloff: float = 0.1) -> np.ndarray:
    """Root-raised-cosine frequency response on the n-point DFT grid (FFT order), unit passband."""
    f = np.abs(np.fft.fftfreq(n, d=1.0 / fs))
    f1 = (1.0 - rolloff) * rs / 2.0
    f2 = (1.0 + rolloff) * rs / 2.0
    H = np.zeros(n, dtype=np.float64)
    H[f <= f1] = 1.0
    band = (f > f1) & (f <= f2)
    H[band] = np.sqrt(0.5 * (1.0 + np.cos(np.pi / (rolloff * rs) * (f[band] - f1))))
    return H


def _bcast(H: np.ndarray, ndim: int, axis: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = H.shape[0]
    return H.reshape(shape)


def tx_shape(symbols: np.ndarray, rho: int, p_watt: np.ndarray | float, rs: float,
             rolloff: float = 0.1, axis: int = -1) -> np.ndarray:
    """Pulse-shaped waveform at rho samples/symbol (Sec. IV-A).

    ``p_watt`` is a scalar or broadcastable per frame (shape of symbols without the time axis).
    """
    s = np.asarray(symbols, dtype=np.complex128)
    axis = axis % s.ndim
    nsym = s.shape[axis]
    n = rho * nsym
    shape = list(s.shape)
    shape[axis] = n
    up = np.zeros(shape, dtype=np.complex128)
    sl = [slice(None)] * s.ndim
    sl[axis] = slice(0, n, rho)
    up[tuple(sl)] = s
    H = _bcast(rrc_response(n, rho * rs, rs, rolloff), s.ndim, axis)
    x = np.fft.ifft(np.fft.fft(up, axis=axis) * H, axis=axis)
    p = np.asarray(p_watt, dtype=np.float64)
    if p.ndim > 0:
        p = np.expand_dims(p, axis)
    return np.sqrt(p) * rho * x


def lpf_decimate(y: np.ndarray, n_out: int, axis: int = -1) -> np.ndarray:
    """Ideal brick-wall low-pass to |f| < f_s,out/2 and resampling to n_out points (Sec. IV-A)."""
    y = np.asarray(y, dtype=np.complex128)
    axis = axis % y.ndim
    n_in = y.shape[axis]
    assert n_out % 2 == 0 and n_out <= n_in
    Y = np.fft.fft(y, axis=axis)
    shape = list(y.shape)
    shape[axis] = n_out
    Z = np.zeros(shape, dtype=np.complex128)
    h = n_out // 2
    src = [slice(None)] * y.ndim
    dst = [slice(None)] * y.ndim
    src[axis] = slice(0, h)
    dst[axis] = slice(0, h)
    Z[tuple(dst)] = Y[tuple(src)]
    src[axis] = slice(n_in - h + 1, n_in)
    dst[axis] = slice(h + 1, n_out)
    Z[tuple(dst)] = Y[tuple(src)]
    return np.fft.ifft(Z, axis=axis) * (n_out / n_in)


def matched_filter_downsample(z: np.ndarray, rho: int, p_watt, rs: float, rolloff: float = 0.1,
                              axis: int = -1) -> np.ndarray:
    """s~ = (1/sqrt(P)) [RRC-filtered z] every rho-th sample from index 0 (the circulant M of Sec. IV-A)."""
    z = np.asarray(z, dtype=np.complex128)
    axis = axis % z.ndim
    n = z.shape[axis]
    H = _bcast(rrc_response(n, rho * rs, rs, rolloff), z.ndim, axis)
    f = np.fft.ifft(np.fft.fft(z, axis=axis) * H, axis=axis)
    sl = [slice(None)] * z.ndim
    sl[axis] = slice(0, n, rho)
    p = np.asarray(p_watt, dtype=np.float64)
    if p.ndim > 0:
        p = np.expand_dims(p, axis)
    return f[tuple(sl)] / np.sqrt(p)


def genie_phase(s_tilde: np.ndarray, s: np.ndarray, axis: int = -1) -> np.ndarray:
    """phi = arg(s^H s~) per frame (Sec. IV-A)."""
    return np.angle(np.sum(np.conj(s) * s_tilde, axis=axis))


def phase_correct(s_tilde: np.ndarray, s: np.ndarray, axis: int = -1) -> np.ndarray:
    phi = genie_phase(s_tilde, s, axis)
    return s_tilde * np.exp(-1j * np.expand_dims(phi, axis))


def mse(s_hat: np.ndarray, s: np.ndarray, axis: int = -1) -> np.ndarray:
    """Per-frame ||s^ - s||^2 / N_sym (Sec. IV-B)."""
    d = s_hat - s
    return np.mean(d.real ** 2 + d.imag ** 2, axis=axis)


def effective_snr_db(s_hat: np.ndarray, s: np.ndarray) -> float:
    """Pooled effective SNR in dB: (number of symbols) / (total squared error), unit-energy symbols."""
    d = s_hat - s
    err = float(np.sum(d.real ** 2 + d.imag ** 2))
    return 10.0 * np.log10(d.size / err)


def rx_loss_and_grad(z: np.ndarray, s: np.ndarray, rho: int, p_watt, rs: float, rolloff: float = 0.1):
    """Mean over frames of the MSE after MF, downsampling and genie phase, and its gradient w.r.t. z.

    The genie phase minimises the loss, so by the envelope theorem it is held
    fixed when differentiating.  Adjoint chain: G_s^ = 2 (s^ - s) / (N_sym F);
    G_s~ = e^{+j phi} G_s^; zero insertion (adjoint of taking every rho-th
    sample); the real RRC response is self-adjoint; divide by sqrt(P).  F is the
    number of frames (mean over frames).  Time axis last.
    """
    z = np.asarray(z, dtype=np.complex128)
    n = z.shape[-1]
    nsym = s.shape[-1]
    nfr = int(np.prod(z.shape[:-1])) if z.ndim > 1 else 1
    st = matched_filter_downsample(z, rho, p_watt, rs, rolloff)
    phi = genie_phase(st, s)
    sh = st * np.exp(-1j * phi[..., None])
    loss = float(np.mean(mse(sh, s)))
    g_sh = 2.0 * (sh - s) / (nsym * nfr)
    g_st = g_sh * np.exp(1j * phi[..., None])
    up = np.zeros(z.shape, dtype=np.complex128)
    up[..., 0:n:rho] = g_st
    H = rrc_response(n, rho * rs, rs, rolloff)
    gz = np.fft.ifft(np.fft.fft(up, axis=-1) * H, axis=-1)
    p = np.asarray(p_watt, dtype=np.float64)
    if p.ndim > 0:
        p = p[..., None]
    return loss, gz / np.sqrt(p)
