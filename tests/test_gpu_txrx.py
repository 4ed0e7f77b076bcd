"""GPU parity of the batched FFT, TX/RX DSP (Sec. IV-A, IV-B), Philox noise and Adam against the oracle."""
import numpy as np
import pytest

import synth
from oracle import philox as PH
from oracle import train as TR
from oracle import txrx as X

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2010_14258_amd import txrx as G  # noqa: E402

DEV = "cuda:0"
RS = 10.7e9


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


@pytest.mark.parametrize("n,npol", [(2, 1), (64, 2), (4096, 1), (8192, 1), (32768, 2), (1 << 20, 1)])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-6)])
def test_fft_matches_numpy(n, npol, dtype, tol):
    print("case: fft", n, npol, dtype, flush=True)
    nw = 3 if n < (1 << 20) else 1
    shape = (nw, n) if npol == 1 else (nw, n, 2)
    x = synth.complex_normal(1, shape)
    ref = np.fft.fft(x, axis=1)
    y = G.fft(_t(x, dtype), npol=npol).cpu().numpy()
    assert _rel(y, ref) <= tol * np.log2(max(n, 2))
    z = G.fft(_t(x, dtype), inverse=True, npol=npol).cpu().numpy()
    assert _rel(z, np.fft.ifft(x, axis=1) * n) <= tol * np.log2(max(n, 2))


@pytest.mark.parametrize("rho,nsym,npol", [(4, 1024, 1), (2, 8192, 1), (4, 8192, 2)])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_tx_lpf_rx_chain(rho, nsym, npol, dtype, tol):
    print("case: txrx", rho, nsym, npol, dtype, flush=True)
    nw = 3
    shape = (nw, nsym) if npol == 1 else (nw, nsym, 2)
    idx = synth.qam16_indices(11, shape)
    p = np.array([1e-3, 2.5e-3, 0.4e-3])
    s = X.qam16(idx)
    x_ref = X.tx_shape(s, rho, p if npol == 1 else p[:, None], RS, axis=1)
    x = G.tx_shape(_t(idx, torch.int32), _t(p, torch.float64), rho, RS, npol=npol, dtype=dtype)
    assert _rel(x.cpu().numpy(), x_ref) <= tol
    # receiver front end: 2 samples/symbol after low-pass filtering and decimation
    nd = 2 * nsym
    r_ref = X.lpf_decimate(x_ref, nd, axis=1)
    r = G.rx_lpf_decimate(_t(x_ref, dtype), nd, npol=npol)
    assert _rel(r.cpu().numpy(), r_ref) <= tol
    # matched filter, genie phase, MSE and its gradient on a distorted waveform
    z = r_ref * np.exp(0.3j) + 0.02 * np.sqrt(p[:, None] if npol == 1 else p[:, None, None]) * synth.complex_normal(
        12, r_ref.shape)
    mse, shat, gz = G.rx_mse(_t(z, dtype), _t(s, dtype), _t(p, torch.float64), 2, RS, npol=npol, want_grad=True,
                             want_shat=True)
    if npol == 1:
        st = X.matched_filter_downsample(z, 2, p, RS)
        sh = X.phase_correct(st, s)
        assert _rel(shat.cpu().numpy(), sh) <= tol
        np.testing.assert_allclose(mse.cpu().numpy(), X.mse(sh, s), rtol=100 * tol)
        _, gref = X.rx_loss_and_grad(z, s, 2, p, RS)
        assert _rel(gz.cpu().numpy(), gref) <= 10 * tol
    else:
        for q in range(2):
            st = X.matched_filter_downsample(z[..., q], 2, p, RS)
            sh = X.phase_correct(st, s[..., q])
            assert _rel(shat.cpu().numpy()[..., q], sh) <= tol
            np.testing.assert_allclose(mse.cpu().numpy()[q::2], X.mse(sh, s[..., q]), rtol=100 * tol)


def test_back_to_back_symbols():
    nsym, rho = 4096, 4
    idx = synth.qam16_indices(13, (2, nsym))
    p = np.array([1e-3, 3e-3])
    x = G.tx_shape(_t(idx, torch.int32), _t(p, torch.float64), rho, RS, dtype=torch.complex128)
    r = G.rx_lpf_decimate(x, 2 * nsym)
    s = G.qam16_symbols(_t(idx, torch.int32), dtype=torch.complex128)
    mse, _, _ = G.rx_mse(r, s, _t(p, torch.float64), 2, RS)
    assert float(mse.max()) < 1e-24


def test_philox_words_bit_exact_and_normals():
    print("case: philox", flush=True)
    w = G.randbits(4 * 1001, seed=0x1234_5678_9ABC, stream_id=77).cpu().numpy().view(np.uint32)
    ref = PH.words(1001, 0x1234_5678_9ABC, 77).astype(np.uint32).reshape(-1)
    np.testing.assert_array_equal(w, ref)
    z = G.randn(4001, seed=5, stream_id=3, dtype=torch.complex128).cpu().numpy()
    np.testing.assert_allclose(z, PH.complex_normal(4001, 5, 3), rtol=0, atol=1e-12)
    z32 = G.randn(4001, seed=5, stream_id=3, dtype=torch.complex64).cpu().numpy()
    np.testing.assert_allclose(z32, PH.complex_normal(4001, 5, 3), rtol=0, atol=1e-5)


def test_adam_matches_oracle_with_mask_and_mirror():
    print("case: adam", flush=True)
    # two symmetric 5-tap filters (complex) with the outer pair of the second masked off
    h = np.concatenate([synth.random_taps(20, [5])[0], synth.random_taps(21, [5])[0]])
    h[0:5] = (h[0:5] + h[0:5][::-1]) / 2
    h[5:10] = (h[5:10] + h[5:10][::-1]) / 2
    mirror = np.array([4, 3, 2, 1, 0, 9, 8, 7, 6, 5], dtype=np.int32)
    maskc = np.array([1, 1, 1, 1, 1, 0, 1, 1, 1, 0], dtype=np.float64)
    h = h * maskc
    theta = _t(h, torch.complex128)
    m = torch.zeros(20, dtype=torch.float64, device=DEV)
    v = torch.zeros_like(m)
    mask = _t(np.repeat(maskc, 2), torch.float64)
    opt = TR.Adam(20)
    th_ref = np.stack([h.real, h.imag], axis=-1).reshape(-1)
    for t in range(1, 6):
        g = synth.random_taps(100 + t, [10])[0]
        G.adam_(theta, _t(g, torch.complex128), m, v, t, mask=mask, mirror=_t(mirror, torch.int32))
        gs = g + g[mirror]
        gs[[2, 7]] = g[[2, 7]]
        gr = np.stack([gs.real, gs.imag], axis=-1).reshape(-1) * np.repeat(maskc, 2)
        th_ref = opt.step(th_ref, gr) * np.repeat(maskc, 2)
    got = torch.view_as_real(theta).cpu().numpy().reshape(-1)
    np.testing.assert_allclose(got, th_ref, rtol=1e-12, atol=1e-15)
    gc = got[0::2] + 1j * got[1::2]
    np.testing.assert_allclose(gc[0:5], gc[0:5][::-1], atol=1e-15)
