"""Pins for the transmitter / receiver oracle (Sec. IV-A, IV-B)."""
import numpy as np
import pytest

import synth
from oracle import txrx as X

RS = 10.7e9


def test_qam16_constellation():
    s = X.qam16(np.arange(16))
    assert len(set(np.round(s * np.sqrt(10), 9))) == 16
    assert abs(np.mean(np.abs(s) ** 2) - 1.0) < 1e-15
    assert set(np.round((s * np.sqrt(10)).real).astype(int)) == {-3, -1, 1, 3}


@pytest.mark.parametrize("rho", [2, 4])
def test_rrc_nyquist(rho):
    # Raised-cosine = |RRC|^2 folded at the symbol rate sums to one (zero ISI).
    nsym = 256
    n = rho * nsym
    H = X.rrc_response(n, rho * RS, RS)
    H2 = (H ** 2).reshape(rho, nsym)
    np.testing.assert_allclose(H2.sum(axis=0), 1.0, atol=1e-12)


@pytest.mark.parametrize("rho_a,rho_d", [(4, 2), (2, 2), (6, 2)])
def test_back_to_back_returns_symbols(rho_a, rho_d):
    nsym = 512
    s = X.qam16(synth.qam16_indices(1, (3, nsym)))
    p = np.array([1e-3, 2e-3, 0.5e-3])
    x = X.tx_shape(s, rho_a, p, RS)
    r = X.lpf_decimate(x, rho_d * nsym)
    st = X.matched_filter_downsample(r, rho_d, p, RS)
    np.testing.assert_allclose(st, s, atol=1e-12)


def test_tx_mean_power():
    nsym = 1 << 14
    s = X.qam16(synth.qam16_indices(2, nsym))
    x = X.tx_shape(s, 4, 2e-3, RS)
    assert abs(np.mean(np.abs(x) ** 2) / 2e-3 - 1) < 0.02


def test_lpf_keeps_band_limited_samples():
    # Decimating a signal that already fits the output band keeps every rho-th sample.
    nsym = 128
    s = X.qam16(synth.qam16_indices(3, nsym))
    x4 = X.tx_shape(s, 4, 1.0, RS)
    x2 = X.lpf_decimate(x4, 2 * nsym)
    np.testing.assert_allclose(x2, x4[::2], atol=1e-13)


def test_awgn_gives_expected_snr():
    nsym = 200000
    s = X.qam16(synth.qam16_indices(4, nsym))
    v = 0.01
    r = s + np.sqrt(v) * synth.complex_normal(5, nsym)
    snr = X.effective_snr_db(X.phase_correct(r, s), s)
    assert abs(snr - 20.0) < 0.05


def test_genie_phase_removes_rotation():
    s = X.qam16(synth.qam16_indices(6, 1000))
    r = s * np.exp(0.7j)
    np.testing.assert_allclose(X.phase_correct(r, s), s, atol=1e-13)


def test_rx_loss_gradient_against_finite_differences():
    nsym, rho = 64, 2
    s = X.qam16(synth.qam16_indices(7, (2, nsym)))
    p = np.array([1e-3, 3e-3])
    z = X.tx_shape(s, rho, p, RS) + 1e-3 * synth.complex_normal(8, (2, rho * nsym))
    loss, gz = X.rx_loss_and_grad(z, s, rho, p, RS)
    eps = 1e-9
    g = synth.rng(9)
    for _ in range(8):
        i, j = int(g.integers(0, 2)), int(g.integers(0, rho * nsym))
        for d in (1.0, 1j):
            zp = z.copy(); zp[i, j] += eps * d
            zm = z.copy(); zm[i, j] -= eps * d
            fd = (X.rx_loss_and_grad(zp, s, rho, p, RS)[0] - X.rx_loss_and_grad(zm, s, rho, p, RS)[0]) / (2 * eps)
            an = gz[i, j].real if d == 1.0 else gz[i, j].imag
            assert abs(fd - an) <= 1e-4 * np.abs(gz).max()
