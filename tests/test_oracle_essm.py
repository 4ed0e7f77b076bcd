"""Pins for the generalised ESSM oracle (Sec. III-D, eq. nl_filtered with per-step filters) and its adjoint."""
import numpy as np
import pytest

import synth
from oracle import essm as E
from oracle import ldbp as O


def _x(seed, shape):
    return synth.complex_normal(seed, shape)


def _eta(seed, kappas, scale=0.4):
    g = synth.rng(seed)
    out = []
    for kap in kappas:
        e = g.uniform(-scale, scale, size=2 * kap + 1)
        e[kap] += 1.0
        out.append(e)
    return out


@pytest.mark.parametrize("npol", [1, 2])
def test_unit_filters_reproduce_ldbp(npol):
    # eta = (1) in every step is the LDBP step: forward and adjoint coincide with oracle.ldbp
    n = 40
    shape = (2, n) if npol == 1 else (2, n, 2)
    x = _x(1, shape)
    taps = synth.random_taps(2, [5, 3, 7], scale=0.5)
    c = synth.random_real(3, 3, -0.4, 0.4)
    eta = [np.ones(1)] * 3
    np.testing.assert_allclose(E.essm_forward(x, taps, c, eta, npol), O.ldbp_forward(x, taps, c, npol), atol=1e-14)
    w = _x(4, shape)
    gx, gt, gc, ge = E.essm_grad(x, taps, c, eta, w, npol)
    rx, rt, rc = O.ldbp_grad(x, taps, c, w, npol)
    np.testing.assert_allclose(gx, rx, atol=1e-12)
    for a, b in zip(gt, rt):
        np.testing.assert_allclose(a, b, atol=1e-12)
    np.testing.assert_allclose(gc, rc, atol=1e-12)
    # d/d eta_0 at eta_0 = 1 equals c dL/dc (phi = c eta_0 P)
    np.testing.assert_allclose([g[0] for g in ge], c * rc, atol=1e-12)


def test_phase_filter_equals_dense_real_circulant():
    # brute force: phi = c E P with the dense circulant matrix of eta (row j: eta_k at column (j-k) mod n)
    n = 9
    u = _x(5, n)
    eta = _eta(6, [3])[0]                  # 2 kappa + 1 = 7 <= n
    P = np.abs(u) ** 2
    np.testing.assert_allclose(E.filter_power(P, eta), E.phase_filter_matrix(eta, n) @ P, atol=1e-14)
    # a filter longer than the waveform wraps around (indices modulo n)
    eta_long = _eta(7, [6])[0]             # 13 > n = 9
    np.testing.assert_allclose(E.filter_power(P, eta_long), E.phase_filter_matrix(eta_long, n) @ P, atol=1e-14)
    c = 0.3
    y = E.filtered_kerr(u, c, eta)
    np.testing.assert_allclose(y, u * np.exp(1j * c * (E.phase_filter_matrix(eta, n) @ P)), atol=1e-14)


def test_constant_envelope_closed_form():
    # |u_j|^2 = A for all j: every phase is c A sum_k eta_k, whatever the filter shape
    n, A = 32, 0.7
    theta = synth.random_real(8, n, -np.pi, np.pi)
    x = np.sqrt(A) * np.exp(1j * theta)
    eta = _eta(9, [4])
    c = np.array([0.45])
    y = E.essm_forward(x, [np.ones(1, dtype=complex)], c, eta)
    np.testing.assert_allclose(y, x * np.exp(1j * c[0] * A * np.sum(eta[0])), atol=1e-14)


def test_zero_coefficients_remove_the_filters():
    n = 30
    x = _x(10, (2, n))
    taps = synth.random_taps(11, [3, 5])
    c = np.zeros(2)
    y = E.essm_forward(x, taps, c, _eta(12, [2, 5]))
    np.testing.assert_allclose(y, O.fir_circular(O.fir_circular(x, taps[0]), taps[1]), atol=1e-13)


def test_coefficient_filter_rescaling_invariance_and_gradient_orthogonality():
    # phi = c (eta * P): (c s, eta / s) leaves the model unchanged, so the loss gradient is orthogonal
    # to that direction: sum_i [c_i dL/dc_i - sum_k eta_k^(i) dL/deta_k^(i)] terms vanish step by step
    n = 36
    x = _x(13, (2, n)) * 0.8
    taps = synth.random_taps(14, [5, 3, 5], scale=0.6)
    c = synth.random_real(15, 3, -0.4, 0.4)
    eta = _eta(16, [2, 3, 1])
    s = np.array([1.7, -0.6, 2.5])
    y0 = E.essm_forward(x, taps, c, eta)
    y1 = E.essm_forward(x, taps, c * s, [e / v for e, v in zip(eta, s)])
    np.testing.assert_allclose(y1, y0, atol=1e-13)
    w = _x(17, (2, n))
    _, _, gc, ge = E.essm_grad(x, taps, c, eta, w)
    for i in range(3):
        assert abs(c[i] * gc[i] - float(np.dot(eta[i], ge[i]))) <= 1e-12 * max(1.0, abs(c[i] * gc[i]))


def _loss(x, taps, c, eta, w, npol=1):
    y = E.essm_forward(x, taps, c, eta, npol)
    return float(np.sum((np.conj(w) * y).real))


@pytest.mark.parametrize("npol", [1, 2])
def test_adjoint_against_central_differences(npol):
    n, Ts, kappas = 29, [5, 3, 7], [2, 0, 3]
    shape = (2, n) if npol == 1 else (2, n, 2)
    x = _x(20, shape) * 0.8
    taps = synth.random_taps(21, Ts, scale=0.5)
    c = synth.random_real(22, len(Ts), -0.3, 0.3)
    eta = _eta(23, kappas)
    w = _x(24, shape)
    gx, gt, gc, ge = E.essm_grad(x, taps, c, eta, w, npol)
    eps = 1e-6
    g = synth.rng(25)
    for _ in range(6):
        idx = tuple(int(g.integers(0, sz)) for sz in shape)
        for d, part in ((1.0, "re"), (1j, "im")):
            xp = x.copy(); xp[idx] += eps * d
            xm = x.copy(); xm[idx] -= eps * d
            fd = (_loss(xp, taps, c, eta, w, npol) - _loss(xm, taps, c, eta, w, npol)) / (2 * eps)
            an = gx[idx].real if part == "re" else gx[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    for i, h in enumerate(taps):
        for k in range(h.shape[0]):
            for d, part in ((1.0, "re"), (1j, "im")):
                tp = [t.copy() for t in taps]; tp[i][k] += eps * d
                tm = [t.copy() for t in taps]; tm[i][k] -= eps * d
                fd = (_loss(x, tp, c, eta, w, npol) - _loss(x, tm, c, eta, w, npol)) / (2 * eps)
                an = gt[i][k].real if part == "re" else gt[i][k].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, k, part)
    for i in range(len(c)):
        cp = c.copy(); cp[i] += eps
        cm = c.copy(); cm[i] -= eps
        fd = (_loss(x, taps, cp, eta, w, npol) - _loss(x, taps, cm, eta, w, npol)) / (2 * eps)
        assert abs(fd - gc[i]) <= 1e-6 * max(1.0, abs(gc[i]))
    for i, e in enumerate(eta):
        for k in range(e.shape[0]):
            ep = [v.copy() for v in eta]; ep[i][k] += eps
            em = [v.copy() for v in eta]; em[i][k] -= eps
            fd = (_loss(x, taps, c, ep, w, npol) - _loss(x, taps, c, em, w, npol)) / (2 * eps)
            assert abs(fd - ge[i][k]) <= 1e-6 * max(1.0, abs(ge[i][k])), (i, k)
