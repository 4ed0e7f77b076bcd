"""Pins for the split-step oracle (Sec. III-A, III-C) against closed forms and invariants."""
import math

import numpy as np
import pytest

import synth
from oracle import ssm as S
from oracle import units as U

ALPHA = U.alpha_from_db_per_km(0.2)
BETA2 = U.beta2_from_ps2_per_km(-21.683)
GAMMA = U.gamma_from_per_w_per_km(1.3)


def _link(**kw):
    base = dict(fs=42.8e9, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=80e3, nspan=1,
                step_len=S.uniform_steps(80e3, 20), edfa_gain=False)
    base.update(kw)
    return S.Link(**base)


def _wave(seed, n, p=1e-3):
    return synth.complex_normal(seed, n) * math.sqrt(p)


def test_linear_limit_closed_form():
    # gamma = 0: u(L) = F^-1 diag(exp(L (j beta2 w^2 / 2 - alpha/2))) F x  (Sec. III-A)
    n = 1024
    link = _link(gamma=0.0, nspan=2)
    x = _wave(1, n)
    y = S.ssm_channel(x, link)
    w = 2 * np.pi * np.fft.fftfreq(n, 1 / link.fs)
    Ltot = 2 * link.span_len
    ref = np.fft.ifft(np.fft.fft(x) * np.exp(Ltot * (1j * BETA2 * w ** 2 / 2 - ALPHA / 2)))
    np.testing.assert_allclose(y, ref, atol=1e-13 * np.abs(ref).max())


def test_nonlinear_limit_closed_form():
    # beta2 = 0 with loss: u(L) = x e^{-alpha L/2} exp(j gamma L_eff(L) |x|^2) for any step split.
    n = 256
    raw = synth.random_real(2, 7, 0.5, 1.5)
    link = _link(beta2=0.0, step_len=[s * 80e3 / raw.sum() for s in raw])
    x = _wave(3, n, p=0.05)
    y = S.ssm_channel(x, link)
    leff = (1 - math.exp(-ALPHA * 80e3)) / ALPHA
    ref = x * math.exp(-ALPHA * 80e3 / 2) * np.exp(1j * GAMMA * leff * np.abs(x) ** 2)
    np.testing.assert_allclose(y, ref, atol=1e-13 * np.abs(ref).max())


def test_energy_conserved_without_loss():
    n = 512
    link = _link(alpha=0.0)
    x = _wave(4, n, p=0.02)
    y = S.ssm_channel(x, link)
    assert abs(np.sum(np.abs(y) ** 2) / np.sum(np.abs(x) ** 2) - 1) < 1e-13


def _soliton_link(nstep, z):
    # Normalised NLSE: beta2 = -1, gamma = 1, alpha = 0; time unit 1, fs = n / window.
    n, window = 1024, 64.0
    return n, window, S.Link(fs=n / window, alpha=0.0, beta2=-1.0, gamma=1.0, span_len=z, nspan=1,
                             step_len=S.uniform_steps(z, nstep), edfa_gain=False)


def test_fundamental_soliton():
    # sech(t) propagates as sech(t) e^{j z / 2} (standard NLSE soliton; Sec. III-A equation with these units).
    z = 4 * math.pi
    n, window, link = _soliton_link(2000, z)
    t = (np.arange(n) - n // 2) * (window / n)
    x = 1 / np.cosh(t)
    ref = x * np.exp(1j * z / 2)
    err_sym = np.max(np.abs(S.ssm_channel_symmetric(x, link) - ref))
    err_asym = np.max(np.abs(S.ssm_channel(x, link) - ref))
    assert err_sym < 1e-4
    assert err_asym < 5e-3


def test_convergence_orders():
    # Sec. III-C: asymmetric SSM error O(1/M), symmetric O(1/M^2).
    z = 2.0
    errs_a, errs_s = [], []
    n, window, fine = _soliton_link(4000, z)
    t = (np.arange(n) - n // 2) * (window / n)
    x = 1.2 / np.cosh(t) * np.exp(0.3j * t)  # not a soliton, so the answer is not trivial
    ref = S.ssm_channel_symmetric(x, fine)
    for m in (25, 100):
        _, _, link = _soliton_link(m, z)
        errs_a.append(np.linalg.norm(S.ssm_channel(x, link) - ref))
        errs_s.append(np.linalg.norm(S.ssm_channel_symmetric(x, link) - ref))
    ra = errs_a[0] / errs_a[1]
    rs = errs_s[0] / errs_s[1]
    assert 3.0 < ra < 5.5, ra
    assert 12.0 < rs < 20.0, rs


def test_dbp_with_identical_steps_inverts_channel():
    n = 2048
    link = _link(nspan=2, edfa_gain=True, step_len=S.uniform_steps(80e3, 10))
    x = _wave(5, n, p=5e-3)
    y = S.ssm_channel(x, link)
    xr = S.fft_dbp(y, link)
    np.testing.assert_allclose(xr, x, atol=1e-12 * np.abs(x).max())


def test_manakov_reduces_to_scalar_for_one_polarisation():
    n = 256
    link1 = _link()
    link2 = _link(npol=2, kerr_scale=1.0)
    x = _wave(6, n, p=0.02)
    xx = np.stack([x, np.zeros_like(x)], axis=-1)
    y2 = S.ssm_channel(xx, link2)
    np.testing.assert_allclose(y2[:, 0], S.ssm_channel(x, link1), atol=1e-15)
    assert np.max(np.abs(y2[:, 1])) == 0.0


def test_ase_noise_is_added_per_span():
    n = 4096
    link = _link(nspan=3, gamma=0.0, beta2=0.0, alpha=0.0, edfa_gain=False, ase_var=2.0)
    x = np.zeros(n, dtype=np.complex128)
    noise = synth.complex_normal(7, (3, n))
    y = S.ssm_channel(x, link, noise)
    np.testing.assert_allclose(y, math.sqrt(2.0) * noise.sum(0), atol=1e-14)


def test_ase_variance_matches_high_gain_limit():
    # For G = e^{alpha L} >> 1 the ASE PSD (G-1) h nu n_sp tends to NF G h nu / 2 (Sec. IV-A definition of n_sp).
    fs = 1e9
    v = U.ase_variance_per_sample(ALPHA, 200e3, 5.0, fs)
    G = math.exp(ALPHA * 200e3)
    approx = U.db_to_lin(5.0) * G * U.PLANCK * U.NU_S / 2 * fs
    assert abs(v / approx - 1) < 1e-3
