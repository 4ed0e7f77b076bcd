"""GPU check of the forward that allocates nothing (ldbp_forward_noalloc, for callers that cannot
allocate): through the C ABI its output equals ldbp_forward's on the same plan, on two calls in a row
(the second smaller, so the static scratch still holds the first call's larger signal), and its guard
flag starts from zero on every call."""
import numpy as np
import pytest

import synth
from oracle import ldbp as O
from tests import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2010_14258_amd import _native as N  # noqa: E402
from paper_2010_14258_amd import ldbp as G  # noqa: E402

DEV = "cuda:0"


def _model(seed, ntap, cscale=0.05, symmetric=False):
    taps = synth.random_taps(seed, ntap, scale=1.0)
    taps = [h / np.sqrt(np.sum(np.abs(h) ** 2)) for h in taps]
    if symmetric:
        taps = [0.5 * (h + h[::-1]) for h in taps]
    c = synth.random_real(seed + 1, len(ntap), -cscale, cscale)
    tp, nt = W.pack_taps(taps)
    return taps, c, torch.from_numpy(tp).to(DEV, torch.complex64), \
        torch.from_numpy(np.asarray(c)).to(DEV, torch.float32), nt


def _case(seed, nwave, n, ntap, plan, symmetric):
    print(f"case: noalloc nwave={nwave} n={n} l={len(ntap)} plan={plan}", flush=True)
    taps, c, tt, ct, nt = _model(seed, ntap, symmetric=symmetric)
    x = synth.complex_normal(seed + 2, (nwave, n)) * 0.5
    xt = torch.from_numpy(x).to(DEV, torch.complex64)
    one = tuple(plan) + (1,)                       # same plan on one stream
    ref = G.ldbp_forward(xt, tt, ct, nt, plan=one)
    y = torch.full_like(xt, complex(float("nan"), 0.0))
    G.ldbp_forward_noalloc(xt, tt, ct, nt, y, plan=plan)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    return x, taps, c, y


def test_noalloc_forward_matches_ldbp_forward_on_two_calls():
    # multi-pass plans, so the intermediate signal lives in the static scratch
    p1 = G.ldbp_forward_plan_query(N.LDBP_C64, 1, 16, 65536, [15] * 50, 0, (10, 1, 7, 1))
    assert p1[0] == 5
    _case(30, 16, 65536, [15] * 50, (10, 1, 7, 1), True)           # 8 MiB of scratch
    x, taps, c, y = _case(40, 3, 10001, [5, 3, 9, 1, 15, 7, 3, 5], (2, 0, 7, 0), False)  # smaller second call
    ref = O.ldbp_forward(x, taps, c)                                # and the oracle on the small case
    got = y.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


def test_noalloc_forward_guard_clears_its_flag():
    taps, c, tt, ct, nt = _model(50, [7] * 6)
    x = torch.from_numpy(synth.complex_normal(51, (2, 4096)) * 0.5).to(DEV, torch.complex64)
    bad = x.clone()
    bad[1, 100] = complex(float("nan"), 0.0)
    y = torch.empty_like(x)
    with pytest.raises(N.LdbpError) as e:
        G.ldbp_forward_noalloc(bad, tt, ct, nt, y, plan=(2, 0, 7, 0), guard=True)
    assert e.value.status == N.LDBP_ENONFINITE
    G.ldbp_forward_noalloc(x, tt, ct, nt, y, plan=(2, 0, 7, 0), guard=True)   # the flag starts at zero again
    ref = G.ldbp_forward(x, tt, ct, nt, plan=(2, 0, 7, 0, 1))
    torch.cuda.synchronize()
    assert torch.equal(y, ref)


def test_noalloc_forward_rejects_a_batch_beyond_its_scratch():
    taps, c, tt, ct, nt = _model(60, [3] * 40)
    n = N.LDBP_NOALLOC_SCRATCH_BYTES // 8 // 2 + 64
    x = torch.zeros((2, n), dtype=torch.complex64, device=DEV)
    y = torch.empty_like(x)
    with pytest.raises(N.LdbpError) as e:
        G.ldbp_forward_noalloc(x, tt, ct, nt, y, plan=(4, 0, 7, 0))
    assert e.value.status == N.LDBP_EWORKSPACE
