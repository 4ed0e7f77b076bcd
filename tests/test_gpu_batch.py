"""GPU parity of batched uneven LDBP inference (one launch, optionally a hipGraph) against the oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import ldbp as O
from tests import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2010_14258_amd import batch as B  # noqa: E402
from paper_2010_14258_amd import ldbp as G  # noqa: E402

DEV = "cuda:0"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _pack(models, waves, dtype):
    taps = np.concatenate([np.concatenate(tp) for tp, _ in models])
    c = np.concatenate([cc for _, cc in models])
    x = np.concatenate(waves, axis=0)
    rd = torch.float32 if dtype == torch.complex64 else torch.float64
    return (torch.from_numpy(taps).to(DEV, dtype), torch.from_numpy(c).to(DEV, rd),
            torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype))


def _mixed(seed, npol=1):
    lengths = [1, 2, 5, 17, 1000, 4099, 7001, 20000, 3, 12345]
    g = synth.rng(seed, 3)
    models, waves = [], []
    for i, n in enumerate(lengths):
        L = int(g.integers(1, 9))
        Ts = [int(t) for t in g.choice([1, 3, 5, 7, 9, 15, 25], size=L)]
        tp = synth.random_taps(seed + 10 + i, Ts)
        tp = [h / np.linalg.norm(h) for h in tp]
        c = synth.random_real(seed + 40 + i, L, -0.3, 0.3)
        models.append((tp, c))
        shape = (n,) if npol == 1 else (n, 2)
        waves.append(synth.complex_normal(seed + 70 + i, shape) * 0.6)
    return lengths, models, waves


@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-12)])
def test_batch_matches_oracle_and_per_waveform_forward(npol, dtype, tol):
    print("case: batch mixed", npol, dtype, flush=True)
    lengths, models, waves = _mixed(5, npol)
    plan = B.BatchPlan(lengths, [len(c) for _, c in models], [len(h) for tp, _ in models for h in tp], dtype=dtype,
                       npol=npol)
    taps, c, x = _pack(models, waves, dtype)
    y = plan.forward(taps, c, x).cpu().numpy()
    off = np.cumsum([0] + lengths)
    for b, (tp, cc) in enumerate(models):
        yb = y[off[b]:off[b + 1]]
        ref = O.ldbp_forward(waves[b], tp, cc, npol=npol)
        assert _rel(yb, ref) <= tol, b
        # the same arithmetic as the single-waveform forward: bit-identical
        xs = torch.from_numpy(waves[b][None]).to(DEV, dtype)
        ts = torch.from_numpy(np.concatenate(tp)).to(DEV, dtype)
        cs = torch.from_numpy(cc).to(DEV, torch.float32 if dtype == torch.complex64 else torch.float64)
        ys = G.ldbp_forward(xs, ts, cs, [len(h) for h in tp], npol=npol).cpu().numpy()[0]
        np.testing.assert_array_equal(yb, ys)


@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-10)])
def test_batch_long_halo_runs_in_several_passes(npol, dtype, tol):
    """A waveform whose total halo (150 steps of 63 taps: 4,650 samples a side) leaves no tile in the
    largest LDS work size runs its steps in groups, one launch per group, beside waveforms that run in
    one pass; each output against the oracle, and the graph replay of the several launches.  The long
    model is the least-squares LDBP of 30 x 100 km at 5 steps per span with 63 taps, each filter
    scaled to unit peak gain (a bounded cascade), on a white input at 0 dBm."""
    print("case: batch several passes", npol, dtype, flush=True)
    g = synth.rng(31, 3)
    lengths = [8000, 3001, 257]
    nsteps = [150, 7, 3]
    models, waves = [], []
    for i, (n, L) in enumerate(zip(lengths, nsteps)):
        if i == 0:
            tp, c = W.ldbp_init(30, 5, 63, kerr_scale=8.0 / 9.0 if npol == 2 else 1.0)
            tp = [W.unit_peak_gain(h) for h in tp]
            amp = math.sqrt(1e-3)
        else:
            Ts = [int(t) for t in g.choice([3, 5, 9, 15], size=L)]
            tp = synth.random_taps(3100 + i, Ts)
            tp = [h / np.linalg.norm(h) for h in tp]
            c = synth.random_real(3200 + i, L, -0.3, 0.3)
            amp = 0.5
        models.append((tp, np.asarray(c, np.float64)))
        shape = (n,) if npol == 1 else (n, 2)
        waves.append(synth.complex_normal(3300 + i, shape) * amp)
    plan = B.BatchPlan(lengths, nsteps, [len(h) for tp, _ in models for h in tp], dtype=dtype, npol=npol)
    taps, c, x = _pack(models, waves, dtype)
    y = plan.forward(taps, c, x)
    yg = torch.empty_like(x)
    for _ in range(2):
        yg.zero_()
        plan.forward(taps, c, x, y=yg, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(yg, y)
    y = y.cpu().numpy()
    off = np.cumsum([0] + lengths)
    for b, (tp, cc) in enumerate(models):
        assert _rel(y[off[b]:off[b + 1]], O.ldbp_forward(waves[b], tp, cc, npol=npol)) <= tol, b


def test_batch_graph_replays():
    print("case: batch graph", flush=True)
    lengths, models, waves = _mixed(6)
    plan = B.BatchPlan(lengths, [len(c) for _, c in models], [len(h) for tp, _ in models for h in tp])
    taps, c, x = _pack(models, waves, torch.complex64)
    ref = plan.forward(taps, c, x).cpu().numpy()
    y = torch.empty_like(x)
    for rep in range(4):
        y.zero_()
        plan.forward(taps, c, x, y=y, graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(y.cpu().numpy(), ref)
        _ = (x * 2).sum().item()   # eager work between replays


def test_batch_symmetric_folded():
    print("case: batch symmetric", flush=True)
    lengths, models, waves = _mixed(7)
    models = [([(h + h[::-1]) / 2 for h in tp], cc) for tp, cc in models]
    plan = B.BatchPlan(lengths, [len(c) for _, c in models], [len(h) for tp, _ in models for h in tp],
                       plan=(0, 0, 9, 1))
    taps, c, x = _pack(models, waves, torch.complex64)
    y = plan.forward(taps, c, x).cpu().numpy()
    off = np.cumsum([0] + lengths)
    for b, (tp, cc) in enumerate(models):
        assert _rel(y[off[b]:off[b + 1]], O.ldbp_forward(waves[b], tp, cc)) <= 1e-4


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 1e-4)])
def test_batch_full_size_uneven_256(dtype, tol):
    """256 waveforms, lengths log-uniform in [4,096, 262,144] (even 5-smooth), 1-25 spans of 100 km,
    2 steps per span, 3/5/7/9 taps per waveform (LS taps at unit peak gain); graph launch; sampled
    outputs vs oracle, and three whole waveforms."""
    print("case: batch full size", dtype, flush=True)
    lengths, nspan, taps_b = W.uneven_batch_spec(401)
    models = W.uneven_models(lengths, nspan, taps_b)
    waves = [W.cd_received(1000 + b, n, ns) for b, (n, ns) in enumerate(zip(lengths, nspan))]
    plan = B.BatchPlan(lengths, [len(c) for _, c in models], [len(h) for tp, _ in models for h in tp], dtype=dtype)
    taps, c, x = _pack(models, waves, dtype)
    y = plan.forward(taps, c, x, graph=True).cpu().numpy().astype(np.complex128)
    off = np.cumsum([0] + lengths)
    g = synth.rng(402)
    for b, (tp, cc) in enumerate(models):
        H = sum((len(h) - 1) // 2 for h in tp)
        n = lengths[b]
        scale = math.sqrt(np.mean(np.abs(y[off[b]:off[b + 1]]) ** 2))
        for m in (0, n - 1, int(g.integers(0, n))):
            ref = O.ldbp_forward(W.cone_sample(waves[b], m, H), tp, cc)[H]
            assert abs(y[off[b] + m] - ref) <= tol * scale, (b, m)
    for b in (0, 100, 255):
        tp, cc = models[b]
        assert _rel(y[off[b]:off[b + 1]], O.ldbp_forward(waves[b], tp, cc)) <= tol
