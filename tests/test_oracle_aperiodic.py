"""Pins for the aperiodic (streaming) oracle: full linear convolution steps, zero and valid edges."""
import numpy as np
import pytest

import synth
from oracle import aperiodic as A
from oracle import essm as OE
from oracle import ldbp as O


def _eta(seed, kappas, scale=0.3):
    g = synth.rng(seed)
    out = []
    for kap in kappas:
        e = g.uniform(-scale, scale, size=2 * kap + 1)
        e[kap] += 1.0
        out.append(e)
    return out


def _brute(x, taps, c, eta=None):
    """Explicit matrices and loops: support grows by K per step; the phase filter sums over the
    support only (P is zero outside it)."""
    cur = np.asarray(x, dtype=np.complex128)
    for i, h in enumerate(taps):
        u = A.toeplitz_full(h, cur.shape[0]) @ cur
        P = np.abs(u) ** 2
        F = np.zeros(P.shape[0])
        for j in range(P.shape[0]):
            if eta is None:
                F[j] = P[j]
                continue
            kap = (len(eta[i]) - 1) // 2
            for k in range(-kap, kap + 1):
                if 0 <= j - k < P.shape[0]:
                    F[j] += eta[i][kap + k] * P[j - k]
        cur = u * np.exp(1j * c[i] * F)
    return cur


@pytest.mark.parametrize("filtered", [False, True])
def test_brute_force_matrices(filtered):
    n = 7
    x = synth.complex_normal(1, n)
    taps = synth.random_taps(2, [3, 5, 1, 3], scale=0.6)
    c = synth.random_real(3, 4, -0.5, 0.5)
    eta = _eta(4, [1, 0, 2, 3]) if filtered else None
    full = _brute(x, taps, c, eta)
    G = sum((len(h) - 1) // 2 for h in taps)
    np.testing.assert_allclose(A.forward_aperiodic(x, taps, c, eta, "zero"), full[G:G + n], atol=1e-13)
    n2 = 31
    x2 = synth.complex_normal(5, n2)
    full2 = _brute(x2, taps, c, eta)
    P = A.halo(taps, eta)
    np.testing.assert_allclose(A.forward_aperiodic(x2, taps, c, eta, "valid"), full2[G + P:G + n2 - P], atol=1e-13)


@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("filtered", [False, True])
def test_zero_edge_is_the_circular_model_on_a_zero_padded_block(npol, filtered):
    n = 40
    shape = (2, n) if npol == 1 else (2, n, 2)
    x = synth.complex_normal(6, shape)
    taps = synth.random_taps(7, [5, 3, 7, 3], scale=0.5)
    c = synth.random_real(8, 4, -0.4, 0.4)
    eta = _eta(9, [2, 1, 0, 3]) if filtered else None
    P = A.halo(taps, eta)
    y = A.forward_aperiodic(x, taps, c, eta, "zero", npol)
    for pad in (P, P + 5):
        xp = A._zpad(x, pad, pad, npol)
        yc = OE.essm_forward(xp, taps, c, eta, npol) if filtered else O.ldbp_forward(xp, taps, c, npol)
        np.testing.assert_allclose(y, A._tslice(yc, pad, pad + n, npol), atol=1e-13)


@pytest.mark.parametrize("filtered", [False, True])
def test_valid_edge_is_the_circular_model_away_from_the_wrap(filtered):
    n = 60
    x = synth.complex_normal(10, (3, n))
    taps = synth.random_taps(11, [7, 5, 3], scale=0.5)
    c = synth.random_real(12, 3, -0.4, 0.4)
    eta = _eta(13, [3, 2, 4]) if filtered else None
    P = A.halo(taps, eta)
    yc = OE.essm_forward(x, taps, c, eta) if filtered else O.ldbp_forward(x, taps, c)
    np.testing.assert_allclose(A.forward_aperiodic(x, taps, c, eta, "valid"), yc[:, P:n - P], atol=1e-13)


def test_linear_cascade_is_one_convolution():
    # c = 0: the stack is one linear convolution with the convolution of all filters (Sec. VI-C)
    n = 50
    x = synth.complex_normal(14, n)
    taps = synth.random_taps(15, [5, 3, 7])
    h = taps[0]
    for t in taps[1:]:
        h = np.convolve(h, t)
    G = (len(h) - 1) // 2
    y = A.forward_aperiodic(x, taps, np.zeros(3), None, "zero")
    np.testing.assert_allclose(y, np.convolve(x, h)[G:G + n], atol=1e-13)


def test_shift_equivariance():
    n, d, e = 30, 9, 4
    x = synth.complex_normal(16, n)
    taps = synth.random_taps(17, [5, 5, 3], scale=0.6)
    c = synth.random_real(18, 3, -0.5, 0.5)
    y = A.forward_aperiodic(x, taps, c, None, "zero")
    yp = A.forward_aperiodic(np.concatenate([np.zeros(d), x, np.zeros(e)]), taps, c, None, "zero")
    np.testing.assert_allclose(yp[d:d + n], y, atol=1e-13)


@pytest.mark.parametrize("filtered", [False, True])
def test_chunked_valid_outputs_reproduce_the_stream(filtered):
    N, B = 200, 37
    x = synth.complex_normal(19, N)
    taps = synth.random_taps(20, [5, 3, 5], scale=0.6)
    c = synth.random_real(21, 3, -0.5, 0.5)
    eta = _eta(22, [2, 3, 1]) if filtered else None
    P = A.halo(taps, eta)
    whole = A.forward_aperiodic(x, taps, c, eta, "zero")
    xe = np.concatenate([np.zeros(P), x, np.zeros(P + B)])  # the stream with zeros beyond its ends
    out = [A.forward_aperiodic(xe[s:s + B + 2 * P], taps, c, eta, "valid") for s in range(0, N, B)]
    np.testing.assert_allclose(np.concatenate(out)[:N], whole, atol=1e-13)
