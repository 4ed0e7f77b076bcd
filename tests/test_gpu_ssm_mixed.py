"""GPU parity of the split-step channel and FFT-DBP (Sec. III-A, IV-A) at lengths 2^a 3^b 5^c against the
oracle: the resident path (n <= 4096) and the mixed-radix passes in LDS, uniform batches and uneven
batch plans (waveforms of different lengths and span counts in one run)."""
import math

import numpy as np
import pytest

import synth
from oracle import design as D
from oracle import ssm as S
from oracle import units as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2010_14258_amd import ssm as G  # noqa: E402

DEV = "cuda:0"
ALPHA = U.alpha_from_db_per_km(0.2)
BETA2 = U.beta2_from_ps2_per_km(-21.683)
GAMMA = U.gamma_from_per_w_per_km(1.3)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _links(fs, nspan, steps, ase_var=0.0, npol=1, span=80e3):
    kw = dict(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=span, nspan=nspan, edfa_gain=True,
              ase_var=ase_var, kerr_scale=8 / 9 if npol == 2 else 1.0)
    return S.Link(step_len=steps, npol=npol, **kw), G.Link(nstep=len(steps), step_len=steps, **kw)


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _wave(seed, nwave, n, npol, p):
    shape = (nwave, n) if npol == 1 else (nwave, n, 2)
    return synth.complex_normal(seed, shape) * math.sqrt(p)


# 3000 and 4050 take the resident path, the others the mixed-radix passes (162000 = 2^4 3^4 5^3,
# 259200 = 2^7 3^4 5^2: rows of 4050 values; 4500 and 6000 have columns of 2 and 3)
CASES = [(3000, 1), (4050, 1), (4500, 1), (6000, 1), (30000, 1), (162000, 1), (259200, 1), (3000, 2), (6000, 2),
         (162000, 2)]


@pytest.mark.parametrize("n,npol", CASES)
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-4)])
def test_channel_parity_mixed_lengths(n, npol, dtype, tol):
    print("case: mixed channel", n, npol, dtype, flush=True)
    fs = 42.8e9
    steps = D.log_steps(80e3, 3, ALPHA)
    var = U.ase_variance_per_sample(ALPHA, 80e3, 5.0, fs)
    o, g = _links(fs, 2, steps, ase_var=var, npol=npol)
    x = _wave(5, 2, n, npol, 5e-3)
    noise = synth.complex_normal(6, (2,) + x.shape)
    ref = S.ssm_channel(x, o, noise)
    y = G.ssm_channel(_t(x, dtype), g, noise=_t(noise, dtype), npol=npol)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("n,npol", CASES)
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-4)])
def test_fft_dbp_parity_mixed_lengths(n, npol, dtype, tol):
    print("case: mixed dbp", n, npol, dtype, flush=True)
    fs = 21.4e9
    steps = D.log_steps(100e3, 3, ALPHA)
    o, g = _links(fs, 3, steps, npol=npol, span=100e3)
    r = _wave(7, 2, n, npol, 5e-3)
    ref = S.fft_dbp(r, o)
    y = G.fft_dbp(_t(r, dtype), g, npol=npol)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), ref) <= tol


def test_mixed_linear_step_closed_form():
    """gamma = 0 over one span: the exact dispersion and loss response exp(z (j beta2 w^2 / 2 - alpha / 2))
    on the DFT grid of a length with factors 3 and 5 (mixed-radix passes)."""
    print("case: mixed closed form", flush=True)
    n, fs = 24000, 21.4e9
    g = G.Link(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=0.0, span_len=50e3, nspan=1, nstep=4, edfa_gain=False)
    x = _wave(9, 1, n, 1, 1e-3)[0]
    w = 2 * np.pi * np.fft.fftfreq(n, 1 / fs)
    ref = np.fft.ifft(np.fft.fft(x) * np.exp(50e3 * (1j * BETA2 * w * w / 2 - ALPHA / 2)))
    y = G.ssm_channel(_t(x[None], torch.complex128), g)
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy()[0], ref) <= 1e-11


def _batch_case(dtype, npol, dbp, tol):
    lens = [4096, 4500, 10000, 6000, 65536, 162000, 3000]
    spans = [1, 3, 2, 4, 1, 2, 3]
    fs = 21.4e9
    steps = D.log_steps(100e3, 2, ALPHA)
    var = 0.0 if dbp else U.ase_variance_per_sample(ALPHA, 100e3, 5.0, fs)
    kw = dict(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=100e3, edfa_gain=True, ase_var=var,
              kerr_scale=8 / 9 if npol == 2 else 1.0)
    plan = G.SsmBatchPlan(lens, spans, G.Link(nspan=1, nstep=len(steps), step_len=steps, **kw), dbp, dtype=dtype,
                          npol=npol)
    assert plan.total_samples == sum(lens)
    assert plan.noise_slots == (0 if dbp else max(spans))
    assert plan.total_sample_steps == sum(n * 2 * s for n, s in zip(lens, spans))
    tail = () if npol == 1 else (2,)
    x = synth.complex_normal(11, (sum(lens),) + tail) * math.sqrt(4e-3)
    noise = synth.complex_normal(12, (max(spans), sum(lens)) + tail) if not dbp else None
    y = plan.run(_t(x, dtype), noise=_t(noise, dtype) if noise is not None else None)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    off = 0
    for n, ns in zip(lens, spans):
        o = S.Link(step_len=steps, npol=npol, nspan=ns, **kw)
        xb = x[off:off + n]
        ref = S.fft_dbp(xb, o) if dbp else S.ssm_channel(xb, o, noise[:ns, off:off + n])
        assert _rel(y[off:off + n], ref) <= tol, (n, ns)
        off += n


@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("dbp", [False, True])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-4)])
def test_uneven_batch_plan_matches_oracle_per_waveform(npol, dbp, dtype, tol):
    print("case: ssm batch plan", npol, dbp, dtype, flush=True)
    _batch_case(dtype, npol, dbp, tol)


def test_uneven_batch_plan_in_place_and_repeatable():
    print("case: ssm batch plan in place", flush=True)
    lens, spans = [4500, 8192, 12000], [2, 1, 3]
    steps = D.log_steps(100e3, 10, ALPHA)
    link = G.Link(fs=21.4e9, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=100e3, nspan=1, nstep=10,
                  step_len=steps)
    plan = G.SsmBatchPlan(lens, spans, link, True)
    x = _t(synth.complex_normal(13, (sum(lens),)) * 0.05, torch.complex64)
    a = plan.run(x)
    b = x.clone()
    plan.run(b, y=b)
    c = plan.run(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("n,npol", [(3, 1), (45, 2), (3000, 1), (4050, 2), (6000, 1), (24000, 2), (162000, 1),
                                    (259200, 1)])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-6)])
def test_mixed_radix_fft_matches_numpy(n, npol, dtype, tol):
    print("case: mixed fft", n, npol, dtype, flush=True)
    from paper_2010_14258_amd import txrx as TX
    shape = (3, n) if npol == 1 else (3, n, 2)
    x = synth.complex_normal(15, shape)
    y = TX.fft(_t(x, dtype), npol=npol).cpu().numpy()
    assert _rel(y, np.fft.fft(x, axis=1)) <= tol * np.log2(n + 1)
    z = TX.fft(_t(x, dtype), inverse=True, npol=npol).cpu().numpy()
    assert _rel(z, np.fft.ifft(x, axis=1) * n) <= tol * np.log2(n + 1)


@pytest.mark.parametrize("rho,nsym,npol", [(6, 1024, 1), (6, 1500, 1), (3, 2000, 2), (6, 8192, 1)])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_tx_rx_at_oversampling_6_and_5_smooth_symbol_counts(rho, nsym, npol, dtype, tol):
    """The transmitter at 3 or 6 samples/symbol (the analog oversampling of Table I) and the receiver
    front end back to 2 samples/symbol, at symbol counts with factors 3 and 5."""
    print("case: tx rx mixed", rho, nsym, npol, dtype, flush=True)
    from oracle import txrx as X
    from paper_2010_14258_amd import txrx as TX
    shape = (3, nsym) if npol == 1 else (3, nsym, 2)
    idx = synth.qam16_indices(17, shape)
    p = np.array([1e-3, 2.5e-3, 0.4e-3])
    s = X.qam16(idx)
    x_ref = X.tx_shape(s, rho, p if npol == 1 else p[:, None], 10.7e9, axis=1)
    x = TX.tx_shape(_t(idx, torch.int32), _t(p, torch.float64), rho, 10.7e9, npol=npol, dtype=dtype)
    assert _rel(x.cpu().numpy(), x_ref) <= tol
    r_ref = X.lpf_decimate(x_ref, 2 * nsym, axis=1)
    r = TX.rx_lpf_decimate(_t(x_ref, dtype), 2 * nsym, npol=npol)
    assert _rel(r.cpu().numpy(), r_ref) <= tol
    mse, _, _ = TX.rx_mse(r, _t(s, dtype), _t(p, torch.float64), 2, 10.7e9, npol=npol)
    assert float(mse.max()) <= 1e-8   # back to back: the receiver returns the symbols
