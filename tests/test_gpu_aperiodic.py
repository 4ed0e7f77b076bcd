"""GPU parity of the aperiodic (streaming) forward against the FP64 oracle, its bit identity with the
periodic forward on padded / cropped blocks, chunked streaming, and argument errors."""
import numpy as np
import pytest

import synth
from oracle import aperiodic as OA
from tests import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2010_14258_amd import _native as N  # noqa: E402
from paper_2010_14258_amd import aperiodic as A  # noqa: E402
from paper_2010_14258_amd import essm as GE  # noqa: E402
from paper_2010_14258_amd import ldbp as G  # noqa: E402

DEV = "cuda:0"
TOL = {torch.complex64: 2e-5, torch.complex128: 1e-12}


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _model(seed, Ts, kappas=None, dtype=torch.complex64, cscale=0.3):
    taps = synth.random_taps(seed, Ts)
    taps = [h / np.linalg.norm(h) for h in taps]
    c = synth.random_real(seed + 1, len(Ts), -cscale, cscale)
    eta = None
    if kappas is not None:
        g = synth.rng(seed + 2)
        eta = []
        for kap in kappas:
            e = g.uniform(-0.3, 0.3, 2 * kap + 1) / max(1, kap)
            e[kap] += 1.0
            eta.append(e)
    rd = torch.float32 if dtype == torch.complex64 else torch.float64
    tp, ntap = W.pack_taps(taps)
    dev = dict(tt=torch.from_numpy(tp).to(DEV, dtype), ct=torch.from_numpy(c).to(DEV, rd), ntap=ntap,
               et=None if eta is None else torch.from_numpy(np.concatenate(eta)).to(DEV, rd),
               nl=None if eta is None else [len(e) for e in eta])
    return taps, c, eta, dev


def _gpu(x, d, edge, npol=1, dtype=torch.complex64, plan=None):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)
    y = A.forward_aperiodic(xt, d["tt"], d["ct"], d["ntap"], edge, d["et"], d["nl"], npol=npol, plan=plan)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("filtered", [False, True])
def test_aperiodic_vs_oracle(dtype, npol, filtered):
    """Zero and valid edges at several plans (one pass, fixed steps per pass, automatic), several tiles."""
    print("case: aperiodic", dtype, npol, filtered, flush=True)
    Ts = [15, 3, 9, 5, 11, 7, 1, 13]
    kappas = [2, 0, 20, 7, 1, 3, 0, 5] if filtered else None
    taps, c, eta, d = _model(40, Ts, kappas, dtype)
    shape = (3, 5003) if npol == 1 else (2, 4001, 2)
    x = synth.complex_normal(41, shape) * 0.6
    for edge in ("zero", "valid"):
        ref = OA.forward_aperiodic(x, taps, c, eta, edge, npol)
        for plan in (None, (1, 0), (3, 0), (8, 0)):
            y = _gpu(x, d, edge, npol, dtype, plan).cpu().numpy().astype(np.complex128)
            assert y.shape == ref.shape
            assert _rel(y, ref) <= TOL[dtype], (edge, plan)


@pytest.mark.parametrize("npol", [1, 2])
def test_short_signals_and_minimal_valid_length(npol):
    print("case: aperiodic short", npol, flush=True)
    Ts = [9, 5, 7]
    taps, c, eta, d = _model(42, Ts, None, torch.complex128)
    P = OA.halo(taps)
    for n in (1, 2, 7, 2 * P + 1, 2 * P + 2):
        shape = (2, n) if npol == 1 else (2, n, 2)
        x = synth.complex_normal(43 + n, shape)
        for edge in ("zero", "valid"):
            if edge == "valid" and n <= 2 * P:
                continue
            ref = OA.forward_aperiodic(x, taps, c, None, edge, npol)
            y = _gpu(x, d, edge, npol, torch.complex128).cpu().numpy()
            assert _rel(y, ref) <= 1e-12, (n, edge)


@pytest.mark.parametrize("filtered", [False, True])
def test_bit_identity_with_the_periodic_forward(filtered):
    """Zero edge = the periodic forward on x padded with P zeros; valid edge = the periodic forward on x
    cropped; same plan, same bits."""
    print("case: aperiodic bits", filtered, flush=True)
    Ts = [15, 9, 15, 5, 15, 7]
    kappas = [3, 20, 0, 2, 5, 1] if filtered else None
    taps, c, eta, d = _model(44, Ts, kappas)
    P = OA.halo(taps, eta)
    x = torch.from_numpy(synth.complex_normal(45, (4, 20011)) * 0.5).to(DEV, torch.complex64)
    for plan in ((2, 0, 0, 0), (0, 0, 0, 0), (3, 0, 9, 0)):
        def per(inp):
            if filtered:
                return GE.essm_forward(inp, d["tt"], d["ct"], d["et"], d["ntap"], d["nl"], plan=plan)
            return G.ldbp_forward(inp, d["tt"], d["ct"], d["ntap"], plan=plan)
        z = A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], "zero", d["et"], d["nl"], plan=plan)
        xp = torch.nn.functional.pad(torch.view_as_real(x), (0, 0, P, P))
        zp = per(torch.view_as_complex(xp.contiguous()))
        v = A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], "valid", d["et"], d["nl"], plan=plan)
        vp = per(x)
        torch.cuda.synchronize()
        assert torch.equal(z, zp[:, P:P + x.shape[1]]), plan
        assert torch.equal(v, vp[:, P:x.shape[1] - P]), plan


@pytest.mark.parametrize("filtered", [False, True])
def test_stream_equalizer_reproduces_the_whole_stream(filtered):
    """Chunks of uneven length pushed through the overlap-save helper give the zero-edge forward of the
    whole stream bit for bit."""
    print("case: stream", filtered, flush=True)
    Ts = [15, 9, 15, 5]
    kappas = [3, 20, 0, 2] if filtered else None
    taps, c, eta, d = _model(46, Ts, kappas)
    N_ = 50000
    x = torch.from_numpy(synth.complex_normal(47, (3, N_)) * 0.5).to(DEV, torch.complex64)
    whole = A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], "zero", d["et"], d["nl"], plan=(2, 0))
    se = A.StreamEqualizer(d["tt"], d["ct"], d["ntap"], d["et"], d["nl"], plan=(2, 0))
    cuts = [0, 5, 7000, 7013, 21000, 21001, 40000, N_]
    outs = [se.push(x[:, a:b]) for a, b in zip(cuts[:-1], cuts[1:])] + [se.flush()]
    got = torch.cat(outs, dim=1)
    torch.cuda.synchronize()
    assert got.shape == whole.shape
    assert torch.equal(got, whole)


def test_large_batch_split_equals_one_stream():
    print("case: aperiodic split", flush=True)
    Ts = [15] * 20
    taps, c, eta, d = _model(48, Ts)
    x = torch.from_numpy(synth.complex_normal(49, (6, 1 << 18)) * 0.5).to(DEV, torch.complex64)
    for edge in ("zero", "valid"):
        a = A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], edge, plan=(4, 0, 0, 0))
        b = A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], edge, plan=(4, 0, 0, 0, 1))
        torch.cuda.synchronize()
        assert torch.equal(a, b), edge


def test_argument_errors():
    taps, c, eta, d = _model(50, [5, 5])
    x = torch.zeros((1, 8), dtype=torch.complex64, device=DEV)   # P = 4: valid needs n > 8
    with pytest.raises(ValueError):
        A.forward_aperiodic(x, d["tt"], d["ct"], d["ntap"], "valid")
    y = torch.empty((1, 1), dtype=torch.complex64, device=DEV)
    lib = N.load()
    st = lib.ldbp_forward_aperiodic(N.LDBP_C64, 1, 1, 8, 2, N.i32_array(d["ntap"]), None, d["tt"].data_ptr(),
                                    d["ct"].data_ptr(), None, x.data_ptr(), y.data_ptr(), N.LDBP_EDGE_VALID, None,
                                    None, 0, None)
    assert st == N.LDBP_EINVAL
    st = lib.ldbp_forward_aperiodic(N.LDBP_C64, 1, 1, 8, 2, N.i32_array(d["ntap"]), None, d["tt"].data_ptr(),
                                    d["ct"].data_ptr(), None, x.data_ptr(), y.data_ptr(), 3, None, None, 0, None)
    assert st == N.LDBP_EINVAL
