"""Pins for the LDBP oracle (eq. model, Sec. III-B) and its adjoint, against definitions other than itself."""
import numpy as np
import pytest

import synth
from oracle import ldbp as O


def _x(seed, shape):
    return synth.complex_normal(seed, shape)


@pytest.mark.parametrize("n,T", [(37, 7), (64, 15), (5, 13), (1, 3), (16, 31)])
def test_fir_equals_fft_circular_convolution(n, T):
    # Asymmetric taps so that a reversed index (correlation instead of convolution) fails.
    x = _x(1, (3, n))
    h = synth.random_taps(2, [T])[0]
    K = (T - 1) // 2
    hpad = np.zeros(n, dtype=np.complex128)
    for k in range(-K, K + 1):
        hpad[k % n] += h[K + k]
    ref = np.fft.ifft(np.fft.fft(x, axis=-1) * np.fft.fft(hpad), axis=-1)
    np.testing.assert_allclose(O.fir_circular(x, h), ref, rtol=0, atol=1e-12)


def test_fir_equals_dense_circulant():
    n, T = 11, 5
    x = _x(3, n)
    h = synth.random_taps(4, [T])[0]
    A = O.circulant_matrix(h, n)
    np.testing.assert_allclose(O.fir_circular(x, h), A @ x, atol=1e-13)
    # A_{m, j} depends only on (m - j) mod n: a circulant.
    for m in range(n):
        np.testing.assert_allclose(np.roll(A[0], m), A[m], atol=0)


def test_full_length_taps_reproduce_frequency_domain_filter():
    # LDBP contains DBP (Sec. III-B): T = n taps from the inverse DFT give the FFT filter exactly.
    n = 33
    K = (n - 1) // 2
    H = np.exp(1j * synth.random_real(5, n, -3, 3))
    m = np.fft.fftfreq(n) * n
    h = np.array([np.sum(H * np.exp(2j * np.pi * m * k / n)) / n for k in range(-K, K + 1)])
    x = _x(6, (2, n))
    ref = np.fft.ifft(np.fft.fft(x, axis=-1) * H, axis=-1)
    np.testing.assert_allclose(O.fir_circular(x, h), ref, atol=1e-12)


def test_linear_only_model_is_one_cascaded_filter():
    # Sec. VI-C: with the nonlinearities removed the model is a single filter, the convolution of all steps.
    n = 64
    taps = synth.random_taps(7, [5, 3, 7])
    x = _x(8, (2, n))
    y = O.ldbp_forward(x, taps, np.zeros(3))
    h = np.convolve(np.convolve(taps[0], taps[1]), taps[2])
    np.testing.assert_allclose(y, O.fir_circular(x, h), atol=1e-12)


def test_kerr_preserves_modulus_and_inverts():
    u = _x(9, (4, 50))
    y = O.kerr(u, 0.37)
    np.testing.assert_allclose(np.abs(y), np.abs(u), atol=1e-14)
    np.testing.assert_allclose(O.kerr(y, -0.37), u, atol=1e-14)
    # Manakov: both polarisations rotated by the same phase c(|ux|^2 + |uy|^2).
    v = _x(10, (3, 20, 2))
    w = O.kerr(v, 0.2, npol=2)
    ph = np.angle(w * np.conj(v))
    np.testing.assert_allclose(ph[..., 0], ph[..., 1], atol=1e-13)
    np.testing.assert_allclose(ph[..., 0], np.angle(np.exp(0.2j * (np.abs(v) ** 2).sum(-1))), atol=1e-13)


def test_remark4_rescaling_invariance():
    # Remark 4: h^(i) -> s h^(i), c_i -> c_i / s^2, h^(i+1) -> h^(i+1) / s leaves f_theta unchanged.
    n = 40
    taps = synth.random_taps(11, [5, 5, 3, 7])
    c = np.array([0.3, -0.2, 0.5, 0.0])
    x = _x(12, (2, n))
    y = O.ldbp_forward(x, taps, c)
    s = 1.7
    t2 = [h.copy() for h in taps]
    c2 = c.copy()
    t2[1] = t2[1] * s
    c2[1] = c2[1] / s ** 2
    t2[2] = t2[2] / s
    np.testing.assert_allclose(O.ldbp_forward(x, t2, c2), y, atol=1e-12)


def _loss(x, taps, c, w, npol=1):
    y = O.ldbp_forward(x, taps, c, npol)
    return float(np.sum((np.conj(w) * y).real))


@pytest.mark.parametrize("npol", [1, 2])
def test_adjoint_against_central_differences(npol):
    n, Ts = 31, [5, 3, 7, 5]
    shape = (2, n) if npol == 1 else (2, n, 2)
    x = _x(13, shape) * 0.8
    taps = synth.random_taps(14, Ts, scale=0.5)
    c = synth.random_real(15, len(Ts), -0.3, 0.3)
    w = _x(16, shape)
    gx, gt, gc = O.ldbp_grad(x, taps, c, w, npol)
    eps = 1e-6
    g = synth.rng(17)
    # input gradient, a few random coordinates, real and imaginary directions
    for _ in range(6):
        idx = tuple(int(g.integers(0, s)) for s in shape)
        for d, part in ((1.0, "re"), (1j, "im")):
            xp = x.copy(); xp[idx] += eps * d
            xm = x.copy(); xm[idx] -= eps * d
            fd = (_loss(xp, taps, c, w, npol) - _loss(xm, taps, c, w, npol)) / (2 * eps)
            an = gx[idx].real if part == "re" else gx[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # every tap
    for i, h in enumerate(taps):
        for k in range(h.shape[0]):
            for d, part in ((1.0, "re"), (1j, "im")):
                tp = [t.copy() for t in taps]; tp[i][k] += eps * d
                tm = [t.copy() for t in taps]; tm[i][k] -= eps * d
                fd = (_loss(x, tp, c, w, npol) - _loss(x, tm, c, w, npol)) / (2 * eps)
                an = gt[i][k].real if part == "re" else gt[i][k].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, k, part, fd, an)
    # every Kerr coefficient
    for i in range(len(c)):
        cp = c.copy(); cp[i] += eps
        cm = c.copy(); cm[i] -= eps
        fd = (_loss(x, taps, cp, w, npol) - _loss(x, taps, cm, w, npol)) / (2 * eps)
        assert abs(fd - gc[i]) <= 1e-6 * max(1.0, abs(gc[i]))


def test_adjoint_dot_product_linear_part():
    # c = 0: y = A x is linear, so Re<A v, w> = Re<v, A^H w> with A^H w the returned input gradient.
    n = 45
    taps = synth.random_taps(18, [7, 3, 9])
    v = _x(19, (3, n))
    w = _x(20, (3, n))
    Av = O.ldbp_forward(v, taps, np.zeros(3))
    gx, _, _ = O.ldbp_grad(v, taps, np.zeros(3), w)
    lhs = np.sum(np.conj(w) * Av)
    rhs = np.sum(np.conj(gx) * v)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_adjoint_orthogonal_to_remark4_direction():
    # The loss is constant along the Remark 4 rescaling curve, so its derivative along it vanishes.
    n = 30
    taps = synth.random_taps(21, [5, 5, 5])
    c = np.array([0.4, -0.3, 0.25])
    x = _x(22, (2, n))
    w = _x(23, (2, n))
    _, gt, gc = O.ldbp_grad(x, taps, c, w)
    # d/ds at s = 1 of (h1 s, c1 / s^2, h2 / s)
    d = np.sum((np.conj(gt[0]) * taps[0]).real) - 2 * c[0] * gc[0] - np.sum((np.conj(gt[1]) * taps[1]).real)
    assert abs(d) <= 1e-10 * (np.abs(gt[0]).sum() + abs(gc[0]) + np.abs(gt[1]).sum())


def test_fold_symmetric_grad():
    gh = np.array([1 + 1j, 2, 3j, 4, 5])
    np.testing.assert_allclose(O.fold_symmetric_grad(gh), [3j, 2 + 4, 1 + 1j + 5])
