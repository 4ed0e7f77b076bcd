"""Time-discretised NLSE, split-step channel and FFT-based DBP (Sec. III-A, Sec. IV-A).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

NLSE (eq. nlse):  du/dz = -(alpha/2) u - j (beta2/2) d^2u/dt^2 + j gamma |u|^2 u.

Discretised (eq. discretized_nlse) with the DFT X_m = sum_k x_k e^{-j 2 pi m k / n}:
  * linear step   D(z): X_m <- X_m exp(z (j beta2 omega_m^2 / 2 - alpha / 2))
    (the solution for gamma = 0, Sec. III-A), omega_m = 2 pi f_m, f_m the DFT
    frequencies.  The printed index rule is off by one at m = n/2; we use the
    standard FFT frequency order (Nyquist bin negative), which is harmless since
    only omega^2 enters.
  * nonlinear step N(z): x <- x exp(j gamma L_eff(z) |x|^2) (Sec. III-A, the
    effective-length form), using the power at the start of the step.

Step order.  The printed asymmetric SSM applies the linear operator first and
the Kerr phase with L_eff after it; with loss that is not exact in the beta2 = 0
limit (the phase would use the attenuated end-of-step power).  We read the
channel step as N(delta) followed by D(delta) -- exact in both limits -- and DBP
as its exact reverse, D^{-1}(delta) followed by N^{-1}(delta), which is also the
sigma(A x) order of eq. (model).

Dual polarisation (Manakov, PMD-free): arrays [..., n, 2], dispersion per
polarisation, phase kerr_scale * gamma L_eff (|x|^2 + |y|^2) on both
(kerr_scale = 8/9 for the Manakov equation).

Pins (tests/test_oracle_ssm.py): gamma = 0 closed form; beta2 = 0 closed form;
energy conservation for alpha = 0; the normalised fundamental soliton; first-
and second-order convergence of the asymmetric and symmetric SSM (Sec. III-C);
DBP with the channel's own steps inverts the channel.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import units


@dataclass
class Link:
    """A fiber link and its split-step discretisation (SI units)."""

    fs: float                      # sampling rate [Hz]
    alpha: float                   # power loss [1/m]
    beta2: float                   # [s^2/m]
    gamma: float                   # [1/(W m)]
    span_len: float                # [m]
    nspan: int
    step_len: Sequence[float]      # per-span step lengths in propagation order [m]
    edfa_gain: bool = True         # multiply by e^{alpha L_sp / 2} after each span
    ase_var: float = 0.0           # per-sample complex noise variance added after each span
    kerr_scale: float = 1.0        # 8/9 for the Manakov equation
    npol: int = 1

    def __post_init__(self):
        self.step_len = [float(s) for s in self.step_len]
        assert abs(sum(self.step_len) - self.span_len) <= 1e-9 * max(1.0, self.span_len)


def uniform_steps(span_len: float, nstep: int) -> list[float]:
    return [span_len / nstep] * nstep


def omega(n: int, fs: float) -> np.ndarray:
    """Angular DFT frequencies 2 pi f_m in FFT order (eq. discretized_nlse)."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / fs)


def _time_axis(npol: int) -> int:
    return -1 if npol == 1 else -2


def lin_response(n: int, z: float, link: Link, inverse: bool = False) -> np.ndarray:
    """exp(z (j beta2 omega^2/2 - alpha/2)) per DFT bin (Sec. III-A); negated exponent for the inverse."""
    w = omega(n, link.fs)
    e = z * (1j * link.beta2 * w * w / 2.0 - link.alpha / 2.0)
    if inverse:
        e = -e
    return np.exp(e)


def lin_step(x: np.ndarray, z: float, link: Link, inverse: bool = False) -> np.ndarray:
    ax = _time_axis(link.npol)
    n = x.shape[ax]
    H = lin_response(n, z, link, inverse)
    if link.npol == 2:
        H = H[:, None]
    X = np.fft.fft(x, axis=ax)
    return np.fft.ifft(X * H, axis=ax)


def _power(x: np.ndarray, npol: int) -> np.ndarray:
    p = x.real * x.real + x.imag * x.imag
    if npol == 2:
        p = p.sum(axis=-1)
    return p


def kerr_step(x: np.ndarray, z: float, link: Link, inverse: bool = False) -> np.ndarray:
    """x exp(+-j kerr_scale gamma L_eff(z) |x|^2) (Sec. III-A)."""
    coef = link.kerr_scale * link.gamma * units.l_eff(z, link.alpha)
    if inverse:
        coef = -coef
    rot = np.exp(1j * coef * _power(x, link.npol))
    if link.npol == 2:
        rot = rot[..., None]
    return x * rot


def ssm_channel(x: np.ndarray, link: Link, noise: Optional[np.ndarray] = None) -> np.ndarray:
    """Split-step propagation over nspan spans with EDFAs (Sec. III-A, Sec. IV-A).

    For each span: every step applies N(delta_j) then D(delta_j); then the EDFA
    multiplies by e^{alpha L_sp/2} (exact loss compensation) and adds ASE.
    ``noise`` (if ase_var > 0) has shape [nspan, *x.shape] with E|w|^2 = 1; it is
    scaled by sqrt(ase_var).
    """
    u = np.asarray(x, dtype=np.complex128).copy()
    gain = np.exp(link.alpha * link.span_len / 2.0)
    for s in range(link.nspan):
        for d in link.step_len:
            u = kerr_step(u, d, link)
            u = lin_step(u, d, link)
        if link.edfa_gain:
            u = u * gain
        if link.ase_var > 0.0:
            assert noise is not None, "ASE requested but no noise supplied"
            u = u + np.sqrt(link.ase_var) * noise[s]
    return u


def ssm_channel_symmetric(x: np.ndarray, link: Link) -> np.ndarray:
    """Symmetric SSM (eq. symmetric_ssm, Sec. III-C): D(delta/2) N(delta) D(delta/2) per step; no EDFA/ASE.

    Only used to pin the convergence order; the channel simulator is the asymmetric form.
    """
    u = np.asarray(x, dtype=np.complex128).copy()
    for s in range(link.nspan):
        for d in link.step_len:
            u = lin_step(u, d / 2.0, link)
            u = kerr_step(u, d, link)
            u = lin_step(u, d / 2.0, link)
    return u


def fft_dbp(r: np.ndarray, link: Link) -> np.ndarray:
    """Frequency-domain digital backpropagation: the exact reverse of ``ssm_channel`` without noise.

    For spans last to first: undo the EDFA gain (e^{-alpha L_sp/2}); then for the
    steps in reverse order apply D^{-1}(delta_j) then N^{-1}(delta_j).  With
    gamma = 0 this is the frequency-domain linear equaliser (Sec. V-B).
    """
    u = np.asarray(r, dtype=np.complex128).copy()
    gain = np.exp(-link.alpha * link.span_len / 2.0)
    for s in range(link.nspan):
        if link.edfa_gain:
            u = u * gain
        for d in reversed(link.step_len):
            u = lin_step(u, d, link, inverse=True)
            u = kerr_step(u, d, link, inverse=True)
    return u
