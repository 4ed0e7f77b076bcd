"""Throughput benchmark of the LDBP hot path on one MI355X.

Workload (default): a batch of 64 received waveforms x 65,536 complex64 samples
(16-QAM, 2 samples/symbol, RRC 0.1, 10.7 GBd, 10 x 100 km), equalised by an
LDBP of l = 50 steps (5 per span, log step sizes) with 15-tap filters and
per-step Kerr coefficients, least-squares initialised.

One timed step = one LDBP forward over the whole batch.  The metric is
samples x steps per second (sum over waveforms of n * l per second), with the
inputs already resident in GPU memory.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 78.6        # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 disabled


def fwd_flops_per_sample_step(T: int) -> int:
    # general complex FIR: T complex multiplies (6 flops) + T-1 complex adds (2) = 8T - 2;
    # Kerr: |u|^2 (3) + c * p (1) + rotation (complex multiply, 6) = 10.  Transcendentals not counted.
    return 8 * T - 2 + 10


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-waves", type=int, default=8, help="waveforms in the oracle's bounded sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2010_14258_amd import ldbp as G
    from paper_2010_14258_amd import _native

    _native.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    nwave, n, L, T = 64, 65536, 50, 15
    # Inputs generated on the GPU: received-like complex Gaussian samples at 4 dBm
    # (mean power 2.5 mW) and 15-tap filters with the magnitude profile of the
    # least-squares inverse-dispersion taps of a 20 km step (unit energy).
    g = torch.Generator(device=dev)
    g.manual_seed(201)
    p = 10 ** ((4.0 - 30) / 10)
    x = (torch.randn((nwave, n), dtype=torch.complex64, device=dev, generator=g) * math.sqrt(p)).contiguous()
    k = torch.arange(-(T // 2), T // 2 + 1, device=dev, dtype=torch.float64)
    xi = 0.0993
    h = torch.exp(1j * (-(k ** 2) / (4 * xi) + math.pi / 4)) * torch.exp(-(k / 6.0) ** 2)
    h = (h / torch.linalg.vector_norm(h)).to(torch.complex64)
    taps = h.repeat(L).contiguous()
    c = torch.full((L,), -1.3e-3 * 8e3, dtype=torch.float32, device=dev)
    ntap = [T] * L
    y = torch.empty_like(x)
    wsz = G.ldbp_forward_workspace_size(x, ntap)
    ws = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)

    stream = torch.cuda.current_stream(dev)

    def step():
        G.ldbp_forward(x, taps, c, ntap, y=y, ws=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    ss = nwave * n * L
    value = ss / (ms_per_step * 1e-3)

    # launches per forward: same pass split the library uses
    from paper_2010_14258_amd._native import load as _load  # noqa: F401
    npass = _passes(L, T)
    launch_ms = ms_per_step / npass
    flops_launch = ss * fwd_flops_per_sample_step(T) / npass
    achieved_tflops = flops_launch / (launch_ms * 1e-3) / 1e12
    bytes_launch = nwave * n * 8 * 2  # read + write one complex64 per sample per pass
    achieved_gbs = bytes_launch / (launch_ms * 1e-3) / 1e9

    out = {
        "metric": "samples*steps/s LDBP forward (equalised waveform samples x LDBP steps per second)",
        "value": value,
        "unit": "samples*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "LDBP inference 64 x 65536 c64, l=50 steps (5/span), 15 taps", "nwave": nwave,
                   "n": n, "steps_l": L, "taps": T, "passes": npass},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_PEAK_TFLOPS, "traffic": None,
                     "hbm_achieved_gbs": achieved_gbs, "hbm_frac": achieved_gbs / HBM_PEAK_GBS,
                     "kernel": "ldbp_fwd_kernel<float,1,8,256>", "launch_ms": launch_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_waves, n, L, T)
    print(json.dumps(out), flush=True)


def _passes(L, T):
    # mirrors the library's default pass split: steps join a pass while 2*halo*8 <= 2048
    K = (T - 1) // 2
    per = max(1, min(64, 2048 // (16 * K))) if K > 0 else 64
    return math.ceil(L / per)


def cpu_baseline(nw, n, L, T):
    """The FP64 oracle (plain NumPy, not tuned) on a bounded sample of the same workload."""
    import synth
    from oracle import ldbp as O

    taps = synth.random_taps(1, [T] * L)
    c = np.full(L, -1e-2)
    x = synth.complex_normal(2, (nw, n)) * 0.05
    t0 = time.perf_counter()
    O.ldbp_forward(x, taps, c)
    dt = time.perf_counter() - t0
    return {"value": nw * n * L / dt, "unit": "samples*steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{nw} of 64 waveforms x {n} samples x {L} steps, FP64 NumPy, single process ({dt:.1f} s)"}


if __name__ == "__main__":
    main()
