"""Throughput benchmark of the LDBP hot path on one MI355X; prints one JSON line.

Workload: 64 received waveforms x 65,536 complex64 samples (16-QAM at 2 samples/symbol, RRC
roll-off 0.1, 10.7 GBd) after 10 x 100 km of fiber with an amplifier per span (NF 5 dB), launch
power 4 dBm.  The waveforms are generated on the GPU by the library itself: Philox symbols, RRC
transmitter at 4 samples/symbol, split-step channel with 100 uniform steps per span and amplifier
noise, brick-wall low-pass and decimation to 2 samples/symbol.  The equaliser is LDBP with
l = 50 steps (5 per span, logarithmic step sizes) of 15-tap filters and per-step Kerr
coefficients, least-squares initialised.

One timed step = one LDBP forward over the whole batch (inputs resident in GPU memory).
value = samples x steps per second = nwave * n * l / time.  Also reported: the per-call time
distribution, forward + backward (block checkpoints every 2 steps), FFT-DBP on the same waveforms
at the smallest steps/span whose effective SNR is within 0.1 dB of LDBP's, one training iteration of
the 32 x 16,384 training configuration, the same forward on 1,024 waveforms (512 MiB per buffer,
beyond the 256 MB last-level cache), the dual-polarisation 8 x 2^20 x 2 configuration (32 x 80 km,
l = 64, 5 shared taps), the 256-waveform uneven batch, the generalised ESSM (every nonlinear step
filtering the power with 41 real taps) forward and forward + backward, overlap-save streaming (the
aperiodic forward on blocks of a continuous stream), the roofline positions of the forward and
backward kernels and the FP64 oracle on the host (one core and all cores of the process's CPU set).

Other --mode values run one part alone (for kernel traces and counters: fwd, pmc, bwd, train, variants,
dbp)
or the training experiments (snr, essm, e1, e8, init), each printing its own JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP32_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz; packed FP32 is not used
NWAVE, NSYM, RHO_A, RHO_D = 64, 32768, 4, 2
NSPAN, SPAN_KM, CH_STEPS = 10, 100.0, 100
LDBP_STPS, TAPS = 5, 15
P_DBM = 4.0
RS = 10.7e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ldbp_fwd_traffic.json")
# Fixed plans of the timed forwards (steps per pass, LDS chunks, outputs per thread, folded symmetric
# filters), so that the kernel traces and counters under profiles/ are of the plan the line reports;
# --autotune times the autotuner's pick instead.
HEADLINE_PLAN = (10, 1, 7, 1)
GENERAL_PLAN = (10, 1, 7, 0)
MANAKOV_PLAN = (16, 2, 3, 1)
BIG_BATCH_PLAN = (10, 1, 7, 1)
BWD_KERNEL_SOURCES = ["paper_2010_14258_amd/csrc/ldbp_bwd.hip", "paper_2010_14258_amd/csrc/ldbp_fir.h",
                      "paper_2010_14258_amd/csrc/ldbp_kernels.h", "paper_2010_14258_amd/csrc/common.h"]
BWD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ldbp_bwd_traffic.json")
KERNEL_SOURCES = ["paper_2010_14258_amd/csrc/ldbp_fwd.hip", "paper_2010_14258_amd/csrc/ldbp_fwd_impl.h",
                  "paper_2010_14258_amd/csrc/ldbp_fir.h",
                  "paper_2010_14258_amd/csrc/common.h"]


def kernel_hash(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fwd_flops_per_sample_step(T: int, folded: bool = False) -> int:
    # general complex FIR: T complex multiplies (6 flops) + T-1 complex additions (2) = 8T - 2;
    # folded symmetric FIR (K = (T-1)/2): K pair additions (2) + K+1 complex multiplies (6) + K
    # complex additions (2) = 10K + 6;
    # Kerr: |u|^2 (3) + c |u|^2 (1) + rotation, a complex multiply (6) = 10; sine/cosine not counted.
    K = (T - 1) // 2
    return (10 * K + 6 if folded else 8 * T - 2) + 10


def bwd_flops_per_sample_step(T: int, folded: bool = False) -> int:
    # the forward step recomputed from the block checkpoint (as above);
    # Kerr adjoint: q = Im(G_y conj y) (3), G_y e^{-j phi} (6), 2 c q (2), times u (2), sum (2),
    # the c-gradient term q |u|^2 (2) = 17;
    # FIR adjoint (correlation with the conjugate taps): the forward FIR count;
    # tap correlation sum_m G_u,m conj(x_{m-k}): a conjugate complex multiply-accumulate (8) per tap,
    # folded: K pair additions (2) and K+1 of them.
    K = (T - 1) // 2
    fir = 10 * K + 6 if folded else 8 * T - 2
    tapcorr = 2 * K + 8 * (K + 1) if folded else 8 * T
    return (fir + 10) + 17 + fir + tapcorr


def event_time(torch, stream, fn, steps: int, warmup: int):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_distribution(torch, stream, fn, reps: int, warmup: int):
    """HIP-event time of each of `reps` calls (ms): median, 10th and 90th percentile."""
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median_ms": float(np.median(t)), "p10_ms": float(np.percentile(t, 10)),
            "p90_ms": float(np.percentile(t, 90)), "calls": reps}


def build_workload(torch, dev, cheap: bool = False, p_dbm: float = P_DBM):
    from paper_2010_14258_amd import init as I
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import txrx as TX

    alpha = I.db_per_km_to_alpha(0.2)
    beta2 = I.ps2_per_km_to_beta2(-21.683)
    gamma = 1.3e-3
    span = SPAN_KM * 1e3
    fs_a, fs_d = RHO_A * RS, RHO_D * RS
    p = torch.full((NWAVE,), I.dbm_to_w(p_dbm), dtype=torch.float64, device=dev)
    words = TX.randbits(NWAVE * NSYM, 201, 0, device=dev).view(NWAVE, NSYM)
    if cheap:
        # kernel-trace and counter runs: same shapes and power, without the channel simulation
        r = TX.randn((NWAVE, RHO_D * NSYM), 203, 0, dtype=torch.complex64, device=dev) * math.sqrt(I.dbm_to_w(p_dbm))
    else:
        x = TX.tx_shape(words, p, RHO_A, RS, dtype=torch.complex64)
        noise = TX.randn((NSPAN,) + tuple(x.shape), 202, 0, dtype=torch.complex64, device=dev)
        ch = SS.Link(fs=fs_a, alpha=alpha, beta2=beta2, gamma=gamma, span_len=span, nspan=NSPAN, nstep=CH_STEPS,
                     edfa_gain=True, ase_var=I.ase_variance(alpha, span, 5.0, fs_a))
        SS.ssm_channel(x, ch, noise=noise, y=x)
        del noise
        r = TX.rx_lpf_decimate(x, RHO_D * NSYM)
        del x
    s = TX.qam16_symbols(words, dtype=torch.complex64)
    taps, c = I.ldbp_parameters(span, NSPAN, LDBP_STPS, TAPS, fs_d, alpha, beta2, gamma)
    taps = [0.5 * (h + h[::-1]) for h in taps]   # the fit of an even response: symmetric up to rounding
    ntap = [len(h) for h in taps]
    tt = torch.from_numpy(np.concatenate(taps)).to(dev, torch.complex64)
    ct = torch.from_numpy(c).to(dev, torch.float32)

    def dbp_link(k):
        return SS.Link(fs=fs_d, alpha=alpha, beta2=beta2, gamma=gamma, span_len=span, nspan=NSPAN, nstep=k,
                       step_len=I.log_step_sizes(span, k, alpha), edfa_gain=True)

    return dict(r=r.contiguous(), s=s, p=p, taps=tt, c=ct, ntap=ntap, dbp_link=dbp_link)


def even_5smooth(v: float) -> int:
    best, bd = 2, float("inf")
    for m in range(max(2, int(v * 0.8)), int(v * 1.25) + 2):
        if m % 2:
            continue
        k = m
        for q in (2, 3, 5):
            while k % q == 0:
                k //= q
        if k == 1 and abs(m - v) < bd:
            best, bd = m, abs(m - v)
    return best


def uneven_batch(torch, dev, reps: int):
    """256 waveforms, lengths log-uniform in [4,096, 262,144] (even 5-smooth), 1-25 spans of 100 km,
    2 steps per span, 3/5/7/9 taps per waveform; one graph-captured launch per batch."""
    import synth
    from paper_2010_14258_amd import batch as BT
    from paper_2010_14258_amd import init as I
    from paper_2010_14258_amd import txrx as TX

    lengths = [even_5smooth(v) for v in synth.log_uniform_lengths(401, 256, 4096, 262144)]
    g = synth.rng(401, 9)
    nspan = g.integers(1, 26, size=256).tolist()
    taps_b = g.choice([3, 5, 7, 9], size=256).tolist()
    alpha = I.db_per_km_to_alpha(0.2)
    beta2 = I.ps2_per_km_to_beta2(-21.683)
    span_model = {}
    taps, cs, nsteps, ntap = [], [], [], []
    for ns, T in zip(nspan, taps_b):
        if T not in span_model:
            tp, c = I.ldbp_parameters(1e5, 1, 2, T, 2 * RS, alpha, beta2, 1.3e-3)
            span_model[T] = ([I.unit_peak_gain(h) for h in tp], c)
        tp, c = span_model[T]
        taps.extend(tp * ns)
        cs.append(np.tile(c, ns))
        nsteps.append(2 * ns)
        ntap.extend([T] * (2 * ns))
    tt = torch.from_numpy(np.concatenate(taps)).to(dev, torch.complex64)
    ct = torch.from_numpy(np.concatenate(cs)).to(dev, torch.float32)
    x = TX.randn((sum(lengths),), 404, 0, device=dev) * math.sqrt(2.5e-3)
    y = torch.empty_like(x)
    best = None
    for plan in [(0, 0, rb, sym) for rb in (7, 9) for sym in (0, 1)]:
        bp = BT.BatchPlan(lengths, nsteps, ntap, plan=plan)
        stream = torch.cuda.current_stream(dev)
        ms = event_time(torch, stream, lambda: bp.forward(tt, ct, x, y=y, graph=True, stream=stream), reps, 2)
        if best is None or ms < best[1]:
            best = (plan, ms, bp.total_sample_steps, bp.total_samples, bp.nitems)
    plan, ms, ss, ns_tot, nitems = best
    # plain FFT-DBP at 10 steps per span on the same inputs: one uneven split-step plan over the batch
    from paper_2010_14258_amd import ssm as SS
    dbp = SS.SsmBatchPlan(lengths, nspan, uneven_dbp_link(10), True)
    yd = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    ms_dbp = event_time(torch, stream, lambda: dbp.run(x, y=yd, stream=stream), max(2, reps // 5), 1)
    return {"value": ss / (ms * 1e-3), "unit": "samples*steps/s", "ms_per_batch": ms, "plan": list(plan),
            "total_samples": ns_tot, "total_sample_steps": ss, "work_items": nitems,
            "equalised_samples_per_s": ns_tot / (ms * 1e-3),
            "fft_dbp_10stps": {"ms_per_batch": ms_dbp, "equalised_samples_per_s": ns_tot / (ms_dbp * 1e-3),
                               "sample_steps": dbp.total_sample_steps,
                               "samples_steps_per_s": dbp.total_sample_steps / (ms_dbp * 1e-3),
                               "ldbp_speedup": ms_dbp / ms},
            "workload": "256 uneven waveforms (4,096-262,144 samples), 2-50 steps, 3-9 taps, one hipGraph launch; "
                        "FFT-DBP at 10 steps/span on the same inputs (mixed-radix passes, one launch pair per step)"}


FFT_LENGTHS = ((65536, 64), (64800, 64), (16384, 256), (15000, 279), (262144, 16), (259200, 16))


def fft_lengths(torch, dev, reps: int):
    """FFT-DBP (10 x 100 km, one step per span) on about 4 M samples per batch at power-of-two lengths
    (register-resident team passes) and at nearby lengths with factors 3 and 5 (mixed-radix passes in
    LDS): time per split step and sample x steps per second."""
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import txrx as TX

    stream = torch.cuda.current_stream(dev)
    link = uneven_dbp_link(1)
    link.nspan = 10
    rows = []
    for n, nw in FFT_LENGTHS:
        x = TX.randn((nw, n), 1, 0, device=dev) * 0.05
        ws = torch.empty(SS.ssm_workspace_size(x, link), dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        ms = event_time(torch, stream, lambda: SS.fft_dbp(x, link, y=y, ws=ws, stream=stream), reps, 2)
        rows.append({"n": n, "nwave": nw, "ms": ms, "us_per_step": ms / 10 * 1e3,
                     "sample_steps_per_s": nw * n * 10 / (ms * 1e-3),
                     "algorithmic_tbs": nw * n * 32 * 10 / (ms * 1e-3) / 1e12})
        del x, y, ws
    return {"mode": "fft_lengths", "rows": rows}


def uneven_dbp_link(steps_per_span: int, fs: float = RHO_D * RS):
    """FFT-DBP link of the uneven batch: 100 km SSMF spans, log step sizes (spans per waveform come
    from the plan)."""
    from paper_2010_14258_amd import init as I
    from paper_2010_14258_amd import ssm as SS
    alpha = I.db_per_km_to_alpha(0.2)
    return SS.Link(fs=fs, alpha=alpha, beta2=I.ps2_per_km_to_beta2(-21.683), gamma=1.3e-3, span_len=1e5, nspan=1,
                   nstep=steps_per_span, step_len=I.log_step_sizes(1e5, steps_per_span, alpha), edfa_gain=True)


def uneven_serving(torch, dev, reps: int, train_iters: int, p_dbm: float = 2.0):
    """The uneven serving batch at equal SNR.  256 waveforms (lengths log-uniform in [4,096, 262,144],
    even 5-smooth; 1-25 spans of 100 km; 3/5/7/9 taps per waveform) of 16-QAM at 10.7 GBd and p_dbm,
    simulated on the GPU: transmitter at 4 samples/symbol, the uneven split-step channel plan (50
    uniform steps per span, amplifier noise), low-pass and decimation to 2 samples/symbol.  LDBP: for
    each tap count one 2-step span model shared by every span, least-squares initialised at unit peak
    gain and trained on a 25-span link (`train_iters` Adam iterations, 8 fixed batches); served as one
    graph-captured launch over the batch.  FFT-DBP: the uneven plan at 1, 2, 3, 5, 10 steps per span.
    Effective SNR pooled over all symbols of the batch."""
    import synth
    from paper_2010_14258_amd import batch as BT
    from paper_2010_14258_amd import init as I
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import train as TRN
    from paper_2010_14258_amd import txrx as TX

    lengths = [even_5smooth(v) for v in synth.log_uniform_lengths(401, 256, 4096, 262144)]
    g = synth.rng(401, 9)
    nspan = g.integers(1, 26, size=256).tolist()
    taps_b = g.choice([3, 5, 7, 9], size=256).tolist()
    alpha = I.db_per_km_to_alpha(0.2)
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    models, train_info = {}, {}
    for T in (3, 5, 7, 9):
        cfg = TRN.TrainConfig(nwave=32, nsym=8192, nspan=25, span_km=100.0, channel_steps=50, ldbp_steps=2,
                              t_init=T, t_final=T, iters=train_iters, powers_dbm=(p_dbm,), tie_spans=True,
                              peak_normalise=True, data_pool=8, seed=410 + T)
        trn = TRN.Trainer(cfg, device=dev)
        snr0 = trn.evaluate(nbatch=1, p_dbm=p_dbm)
        trn.train(train_iters)
        snr1 = trn.evaluate(nbatch=1, p_dbm=p_dbm)
        models[T] = (trn.taps.clone(), trn.c.clone())
        train_info[T] = {"init_snr_db_25_spans": snr0, "trained_snr_db_25_spans": snr1}
        del trn
    train_s = time.perf_counter() - t0
    # the received batch
    fs_a = RHO_A * RS
    xa = []
    p_w = torch.full((1,), I.dbm_to_w(p_dbm), dtype=torch.float64, device=dev)
    syms = []
    for b, n in enumerate(lengths):
        words = TX.randbits(n // 2, 402, b, device=dev).view(1, n // 2)
        xa.append(TX.tx_shape(words, p_w, RHO_A, RS).view(-1))
        syms.append(TX.qam16_symbols(words))
    xa = torch.cat(xa)
    ch_link = SS.Link(fs=fs_a, alpha=alpha, beta2=I.ps2_per_km_to_beta2(-21.683), gamma=1.3e-3, span_len=1e5,
                      nspan=1, nstep=50, edfa_gain=True, ase_var=I.ase_variance(alpha, 1e5, 5.0, fs_a))
    ch = SS.SsmBatchPlan([2 * n for n in lengths], nspan, ch_link, False)
    noise = TX.randn((ch.noise_slots, xa.numel()), 403, 0, device=dev)
    ch.run(xa, y=xa, noise=noise)
    del noise, ch
    r, off = [], 0
    for n in lengths:
        r.append(TX.rx_lpf_decimate(xa[off:off + 2 * n].view(1, 2 * n), n).view(-1))
        off += 2 * n
    r = torch.cat(r)
    del xa
    torch.cuda.empty_cache()

    def snr(z):
        """Pooled SNR over the batch and per tap count of the LDBP models (waveforms grouped as served)."""
        err, cnt, o = {}, {}, 0
        for n, s, T in zip(lengths, syms, taps_b):
            mse, _, _ = TX.rx_mse(z[o:o + n].view(1, n), s, p_w, RHO_D, RS)
            e = float(mse.sum().item()) * (n // 2)
            for key in ("all", str(T)):
                err[key] = err.get(key, 0.0) + e
                cnt[key] = cnt.get(key, 0) + n // 2
            o += n
        return {key: 10.0 * math.log10(cnt[key] / err[key]) for key in err}

    # LDBP serving plan with the trained span models
    taps, cs, nsteps, ntap = [], [], [], []
    for ns, T in zip(nspan, taps_b):
        tt, cc = models[T]
        taps.append(tt.repeat(ns))
        cs.append(cc.repeat(ns))
        nsteps.append(2 * ns)
        ntap.extend([T] * (2 * ns))
    tt, ct = torch.cat(taps), torch.cat(cs)
    bp = BT.BatchPlan(lengths, nsteps, ntap, plan=(0, 0, 7, 1))
    y = torch.empty_like(r)
    ms_ldbp = event_time(torch, stream, lambda: bp.forward(tt, ct, r, y=y, graph=True, stream=stream), reps, 2)
    snr_ldbp_groups = snr(bp.forward(tt, ct, r, graph=False))
    snr_ldbp = snr_ldbp_groups["all"]
    sweep, sweep_groups, times = {}, {}, {}
    for k in (1, 2, 3, 5, 10):
        dp = SS.SsmBatchPlan(lengths, nspan, uneven_dbp_link(k), True)
        yd = dp.run(r)
        sweep_groups[k] = snr(yd)
        sweep[k] = sweep_groups[k]["all"]
        times[k] = event_time(torch, stream, lambda: dp.run(r, y=yd, stream=stream), max(2, reps // 5), 1)
        del dp
    k, equal = pick_dbp_setting(sweep, snr_ldbp)
    ns_tot = sum(lengths)
    return {"mode": "uneven_snr", "launch_dbm": p_dbm, "total_samples": ns_tot,
            "ldbp": {"snr_db": snr_ldbp, "ms_per_batch": ms_ldbp, "equalised_samples_per_s": ns_tot / (ms_ldbp * 1e-3),
                     "sample_steps": bp.total_sample_steps, "plan": [0, 0, 7, 1]},
            "ldbp_snr_db_by_taps": {g: v for g, v in snr_ldbp_groups.items() if g != "all"},
            "fft_dbp": {str(kk): {"snr_db": sweep[kk], "ms_per_batch": times[kk],
                                  "snr_db_by_taps_group": {g: v for g, v in sweep_groups[kk].items() if g != "all"},
                                  "equalised_samples_per_s": ns_tot / (times[kk] * 1e-3)} for kk in sweep},
            "fft_dbp_steps_per_span_at_equal_snr": k, "fft_dbp_reaches_ldbp_snr": equal,
            ("ldbp_speedup_at_equal_snr" if equal else "ldbp_speedup_vs_best_fft_dbp_unequal_snr"): times[k] / ms_ldbp,
            "ldbp_speedup_vs_fft_dbp_10stps": times[10] / ms_ldbp,
            "span_models": train_info, "train_s": train_s, "train_iters": train_iters,
            "workload": "256 uneven waveforms (4,096-262,144 samples, 1-25 x 100 km, 3/5/7/9 taps, 2 steps/span), "
                        "GPU-simulated 16-QAM"}


def big_batch(torch, dev, W, reps: int):
    """The inference forward on 1,024 waveforms (the 64 received waveforms repeated 16 times): 512 MiB
    per buffer, so input and output no longer fit the 256 MB last-level cache."""
    from paper_2010_14258_amd import ldbp as L

    r = W["r"].repeat(16, 1)
    taps, c, ntap = W["taps"], W["c"], W["ntap"]
    nwave, n = r.shape
    stream = torch.cuda.current_stream(dev)
    plan = BIG_BATCH_PLAN
    y = torch.empty_like(r)
    ws = torch.empty(max(L.ldbp_forward_workspace_size(r, ntap, plan=plan), 1), dtype=torch.uint8, device=dev)
    ms = event_time(torch, stream, lambda: L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan, ws=ws, stream=stream),
                    reps, 2)
    npass = L.ldbp_forward_plan_query(0, 1, nwave, n, ntap, plan=plan)[0]
    ss = nwave * n * len(ntap)
    flops = nwave * n * sum(fwd_flops_per_sample_step(t, bool(plan[3])) for t in ntap)
    moved = npass * nwave * n * 16
    return {"nwave": nwave, "n": n, "plan": list(plan), "passes": npass, "ms": ms, "value": ss / (ms * 1e-3),
            "unit": "samples*steps/s", "achieved_tflops": flops / (ms * 1e-3) / 1e12,
            "alu_frac": flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
            "algorithmic_hbm_gbs": moved / (ms * 1e-3) / 1e9, "hbm_frac": moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


ROOF_STEPS_PER_PASS = (1, 2, 3, 4, 6, 10)


def roof_sweep(torch, dev, W, reps: int, warmup: int):
    """The 1,024-waveform forward (folded 15-tap filters, l = 50) at each steps-per-pass count of
    ROOF_STEPS_PER_PASS, one stream: time per forward and per launch, algorithmic HBM bytes (read and
    write every sample once per pass) and flops per second."""
    from paper_2010_14258_amd import ldbp as L

    r = W["r"].repeat(16, 1)
    taps, c, ntap = W["taps"], W["c"], W["ntap"]
    nwave, n = r.shape
    stream = torch.cuda.current_stream(dev)
    y = torch.empty_like(r)
    rows = []
    flops = nwave * n * sum(fwd_flops_per_sample_step(t, True) for t in ntap)
    for S in ROOF_STEPS_PER_PASS:
        plan = (S, 1, 7, 1, 1)
        ws = torch.empty(max(L.ldbp_forward_workspace_size(r, ntap, plan=plan), 1), dtype=torch.uint8,
                         device=dev)
        ms = event_time(torch, stream, lambda: L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan, ws=ws,
                                                              stream=stream), reps, warmup)
        npass, tile_len, _ = L.ldbp_forward_plan_query(0, 1, nwave, n, ntap, plan=plan)
        moved = npass * nwave * n * 16
        rows.append({"steps_per_pass": S, "plan": list(plan[:4]), "passes": npass, "tile_len": tile_len,
                     "ms": ms, "us_per_launch": ms / npass * 1e3,
                     "value": nwave * n * len(ntap) / (ms * 1e-3),
                     "algorithmic_bytes_per_launch": nwave * n * 16,
                     "algorithmic_hbm_gbs": moved / (ms * 1e-3) / 1e9,
                     "hbm_frac": moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                     "alu_frac": flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS})
        del ws
    return {"nwave": nwave, "n": n, "steps_l": len(ntap), "taps": TAPS, "rows": rows}


def manakov(torch, dev, reps: int):
    """Dual polarisation: 8 waveforms x 2^20 samples x 2 polarisations (524,288 16-QAM symbols per
    polarisation), 32 x 80 km, PMD-free Manakov channel (Kerr phase 8/9 gamma (|x|^2 + |y|^2)) with 10
    uniform steps per span and amplifier noise, LDBP l = 64 (2 steps per span) with 5 taps shared by
    both polarisations.  Forward and forward + backward."""
    from paper_2010_14258_amd import init as I
    from paper_2010_14258_amd import ldbp as L
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import txrx as TX

    nw, nsym, nspan, span = 8, 524288, 32, 80e3
    alpha = I.db_per_km_to_alpha(0.2)
    beta2 = I.ps2_per_km_to_beta2(-21.683)
    gamma = 1.3e-3
    fs_a, fs_d = RHO_A * RS, RHO_D * RS
    p_w = I.dbm_to_w(2.0)
    p = torch.full((nw,), p_w, dtype=torch.float64, device=dev)
    words = TX.randbits(nw * nsym * 2, 501, 0, device=dev).view(nw, nsym, 2)
    x = TX.tx_shape(words, p, RHO_A, RS, npol=2, dtype=torch.complex64)
    ch = SS.Link(fs=fs_a, alpha=alpha, beta2=beta2, gamma=gamma, span_len=span, nspan=nspan, nstep=10,
                 edfa_gain=True, ase_var=I.ase_variance(alpha, span, 5.0, fs_a), kerr_scale=8.0 / 9.0)
    noise = TX.randn((nspan,) + tuple(x.shape), 502, 0, dtype=torch.complex64, device=dev)
    SS.ssm_channel(x, ch, noise=noise, y=x, npol=2)
    del noise
    r = TX.rx_lpf_decimate(x, RHO_D * nsym, npol=2).contiguous()
    del x
    torch.cuda.empty_cache()
    tp, cc = I.ldbp_parameters(span, nspan, 2, 5, fs_d, alpha, beta2, gamma, kerr_scale=8.0 / 9.0)
    tp = [0.5 * (h + h[::-1]) for h in tp]
    ntap = [len(h) for h in tp]
    taps = torch.from_numpy(np.concatenate(tp)).to(dev, torch.complex64)
    c = torch.from_numpy(cc).to(dev, torch.float32)
    ell = len(ntap)
    n = r.shape[1]
    stream = torch.cuda.current_stream(dev)
    plan = MANAKOV_PLAN
    y = torch.empty_like(r)
    ws = torch.empty(max(L.ldbp_forward_workspace_size(r, ntap, 2, plan=plan), 1), dtype=torch.uint8, device=dev)
    ms = event_time(torch, stream,
                    lambda: L.ldbp_forward(r, taps, c, ntap, npol=2, y=y, plan=plan, ws=ws, stream=stream), reps, 2)
    S = 2   # the library's default block length
    ck = torch.empty((L.num_checkpoints(ell, S),) + tuple(r.shape), dtype=r.dtype, device=dev)
    z = L.ldbp_forward(r, taps, c, ntap, npol=2)
    s = TX.qam16_symbols(words, dtype=torch.complex64)
    mse, _, gy = TX.rx_mse(z, s, p, RHO_D, RS, npol=2, want_grad=True)
    bws = torch.empty(L.ldbp_backward_workspace_size(r, ntap, 2, ckpt=ck, ckpt_every=S), dtype=torch.uint8,
                      device=dev)

    def fwd_bwd():
        L.ldbp_forward(r, taps, c, ntap, npol=2, y=y, ckpt=ck, ckpt_every=S, plan=(0, 0, 0, 1), stream=stream)
        L.ldbp_backward(r, taps, c, ntap, gy, npol=2, ckpt=ck, ckpt_every=S, need_gx=False, symmetric=True, ws=bws,
                        stream=stream)

    ms_fb = event_time(torch, stream, fwd_bwd, max(3, reps // 3), 1)
    ss = nw * n * ell
    return {"workload": "8 waveforms x 1,048,576 samples x 2 polarisations, 32 x 80 km Manakov, l = 64, 5 shared taps",
            "plan": list(plan), "fwd_ms": ms, "fwd_time_samples_steps_per_s": ss / (ms * 1e-3),
            "fwd_pol_samples_steps_per_s": 2 * ss / (ms * 1e-3), "fwd_bwd_ms": ms_fb,
            "fwd_bwd_time_samples_steps_per_s": ss / (ms_fb * 1e-3), "ckpt_every": S,
            "launch_dbm_per_pol": 2.0,
            "ls_init_snr_db": 10.0 * math.log10(1.0 / float(mse.mean().item())),
            "note": "the timing does not depend on the filter values; 5-tap least-squares filters do not equalise "
                    "this link before training (their gain above one outside the signal band compounds over 64 "
                    "steps), so the LS-initialised SNR is not a quality figure"}


def equal_snr_trained(torch, dev, iters: int, powers, reps: int, variants=((25, 3),), data_pool: int = 0,
                      lr_schedule: str = "constant"):
    """The equal-SNR comparison with a trained model: LDBP (l = 50, 5 steps per span) trained by the
    training recipe (32 x 16,384 waveforms per batch simulated on the GPU, launch powers {2, 3, 4} dBm,
    filters pruned from 25 to 3 taps, Adam), then evaluated at each launch power on the 64 x 65,536
    inference batch against FFT-DBP at 1-20 steps per span; the FFT-DBP setting compared is the
    smallest with SNR >= SNR_LDBP - 0.1 dB.  lr_schedule "cosine": Adam's step size decays from 1e-3 to
    1e-4 by a half cosine after the last pruning event."""
    from paper_2010_14258_amd import autotune as AT
    from paper_2010_14258_amd import ldbp as L
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import train as TRN
    from paper_2010_14258_amd import txrx as TX

    models = []
    for t_init, t_final in variants:
        trn = TRN.Trainer(TRN.TrainConfig(iters=iters, t_init=t_init, t_final=t_final, data_pool=data_pool,
                                          lr_schedule=lr_schedule), device=dev)
        t0 = time.perf_counter()
        curve = []
        for it in range(iters):
            loss = trn.step(sync=(it + 1) % 250 == 0)
            if (it + 1) % 250 == 0:
                curve.append([it + 1, loss, int(sum(trn.ntap))])
                print(f"train {t_init}->{t_final} {it + 1}/{iters} loss {loss:.4e} taps {sum(trn.ntap)} "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        models.append({"taps_init": t_init, "taps_final": t_final, "train_seconds": time.perf_counter() - t0,
                       "loss_curve": curve, "taps": trn.taps.contiguous(), "c": trn.c.contiguous(),
                       "ntap": list(trn.ntap)})
        del trn
    # the least-squares models (the method without learning) at each model's initial and final length
    ls = {}
    for T in sorted({t for v in variants for t in v}):
        trn = TRN.Trainer(TRN.TrainConfig(iters=1, t_init=T, t_final=T), device=dev)
        ls[T] = (trn.taps.contiguous(), trn.c.contiguous(), list(trn.ntap))
        del trn
    stream = torch.cuda.current_stream(dev)
    out_models = [{k: v for k, v in m.items() if k not in ("taps", "c", "ntap")} | {"total_taps": int(sum(m["ntap"]))}
                  for m in models]
    rows = []
    for (mi, m), p_dbm in [(mm, p) for p in powers for mm in enumerate(models)]:
        taps, c, ntap = m["taps"], m["c"], m["ntap"]
        W = build_workload(torch, dev, p_dbm=p_dbm)
        r = W["r"]
        y = torch.empty_like(r)
        z = L.ldbp_forward(r, taps, c, ntap, plan=(0, 0, 0, 1))
        snr_tr = snr_db(TX, z, W["s"], W["p"])
        snr_ls = snr_db(TX, L.ldbp_forward(r, W["taps"], W["c"], W["ntap"], plan=(0, 0, 0, 1)), W["s"], W["p"])
        snr_ls_init = {str(T): snr_db(TX, L.ldbp_forward(r, *ls[T], plan=(0, 0, 0, 1)), W["s"], W["p"])
                       for T in (m["taps_init"], m["taps_final"])}
        sweep = {}
        for k in (1, 2, 3, 5, 10, 20):
            sweep[k] = snr_db(TX, SS.fft_dbp(r, W["dbp_link"](k)), W["s"], W["p"])
        k, equal = pick_dbp_setting(sweep, snr_tr)
        plan, _, _ = AT.tune_forward(r, taps, c, ntap, symmetric=True, reps=3)
        ws = torch.empty(max(L.ldbp_forward_workspace_size(r, ntap, plan=plan), 1), dtype=torch.uint8, device=dev)
        ms_l = event_time(torch, stream, lambda: L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan, ws=ws,
                                                                stream=stream), reps, 2)
        link = W["dbp_link"](k)
        dws = torch.empty(SS.ssm_workspace_size(r, link), dtype=torch.uint8, device=dev)
        ms_d = event_time(torch, stream, lambda: SS.fft_dbp(r, link, y=y, ws=dws, stream=stream), max(3, reps // 3), 1)
        rows.append({"model": mi, "launch_dbm": p_dbm, "ldbp_trained_snr_db": snr_tr, "ldbp_ls_init_snr_db": snr_ls,
                     "ldbp_ls_snr_db_by_taps": snr_ls_init,
                     "fft_dbp_snr_db_by_steps_per_span": sweep, "fft_dbp_steps_per_span": k,
                     "fft_dbp_reaches_ldbp_snr": equal, "ldbp_ms": ms_l, "fft_dbp_ms": ms_d,
                     "ldbp_plan": list(plan),
                     ("ldbp_speedup_at_equal_snr" if equal else "ldbp_speedup_vs_best_fft_dbp_unequal_snr"):
                         ms_d / ms_l})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del W, r, y, z
        torch.cuda.empty_cache()
    return {"workload": "64 waveforms x 65,536 c64 samples, 10 x 100 km, LDBP l = 50 (5 steps per span) trained",
            "train_iterations": iters, "lr_schedule": lr_schedule, "models": out_models, "by_power": rows}


def manakov_trained(torch, dev, iters: int, powers, pool: int = 4, channel_steps: int = 25):
    """Training of the dual-polarisation configuration: 8 waveforms x 2^20 samples x 2 polarisations per
    batch (independent 16-QAM per polarisation, 2 samples/symbol), 32 x 80 km PMD-free Manakov channel
    simulated at 4 samples/symbol with `channel_steps` uniform steps per span and amplifier noise;
    LDBP l = 64 (2 steps per span), 5 taps shared by both polarisations, least-squares filters at unit
    peak gain.  The channel simulation of a batch costs about as much as 30 training iterations, so
    training cycles through a fixed pool of `pool` batches (32 M symbols); SNRs are measured on held-out
    batches.  Adam's step size decays from 1e-3 to 1e-4 by a half cosine over the run.  Reports the
    initial and trained SNR per power, FFT-DBP at 1, 2 and 4 steps per span on the same held-out
    waveforms, and the training time."""
    from paper_2010_14258_amd import train as TRN

    cfg = TRN.TrainConfig(nwave=8, nsym=524288, nspan=32, span_km=80.0, channel_steps=channel_steps,
                          ldbp_steps=2, t_init=5, t_final=5, iters=iters, powers_dbm=tuple(powers), npol=2,
                          peak_normalise=True, data_pool=pool, ckpt_every=2, seed=501, lr=1e-3,
                          lr_schedule="cosine", lr_final=1e-4)
    trn = TRN.Trainer(cfg, device=dev)
    init = {p_: trn.evaluate(nbatch=1, p_dbm=p_) for p_ in powers}
    dbp = {p_: {k: trn.evaluate_fft_dbp(k, nbatch=1, p_dbm=p_) for k in (1, 2, 4)} for p_ in powers}
    for it in range(pool):                # simulate the pool before the clock starts
        trn.train_batch(it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = []
    for it in range(iters):
        loss = trn.step(sync=(it + 1) % 250 == 0)
        if (it + 1) % 250 == 0:
            curve.append([it + 1, loss])
            print(f"manakov train {it + 1}/{iters} loss {loss:.4e} {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    trained = {p_: trn.evaluate(nbatch=1, p_dbm=p_) for p_ in powers}
    return {"mode": "manakov_train",
            "workload": "8 x 1,048,576 x 2 pol, 32 x 80 km Manakov, l = 64 (2 steps/span), 5 shared taps",
            "iters": iters, "pool_batches": pool, "channel_steps_per_span": channel_steps,
            "adam_lr": "1e-3 to 1e-4, half cosine",
            "train_s": train_s, "ms_per_iteration": train_s / iters * 1e3,
            "ls_unit_peak_init_snr_db": init, "trained_snr_db": trained, "fft_dbp_snr_db": dbp,
            "loss_curve": curve, "held_out": "1 batch per power (8 x 524,288 x 2 symbols) from seeds not trained on"}


def essm_timing(torch, dev, W, reps: int, kappa: int = 20, plan=None):
    """The generalised ESSM on the inference workload: the same l = 50 steps of 15 folded taps, every
    nonlinear step filtering the power with 2 kappa + 1 real taps.  Forward (autotuned plan) and forward
    with checkpoints every 2 steps + backward.  The filters are unit filters padded with zeros (the
    time does not depend on the values), so the output must equal the LDBP forward's."""
    from paper_2010_14258_amd import autotune as AT
    from paper_2010_14258_amd import essm as E
    from paper_2010_14258_amd import ldbp as L
    from paper_2010_14258_amd import txrx as TX

    r, taps, c, ntap = W["r"], W["taps"], W["c"], W["ntap"]
    nwave, n = r.shape
    ell, ne = len(ntap), 2 * kappa + 1
    eta_np = np.zeros((ell, ne), dtype=np.float32)
    eta_np[:, kappa] = 1.0
    eta = torch.from_numpy(eta_np.reshape(-1)).to(dev)
    nl = [ne] * ell
    stream = torch.cuda.current_stream(dev)
    if plan is None:
        plan, _, _ = AT.tune_forward(r, taps, c, ntap, symmetric=True, reps=3, eta=eta, nl_ntap=nl)
    y = torch.empty_like(r)
    ws = torch.empty(max(E.essm_forward_workspace_size(r, ntap, nl, plan=plan), 1), dtype=torch.uint8, device=dev)
    ms = event_time(torch, stream,
                    lambda: E.essm_forward(r, taps, c, eta, ntap, nl, y=y, plan=plan, ws=ws, stream=stream), reps, 2)
    npass, tile_len, spp = E.essm_forward_plan_query(0, 1, nwave, n, ntap, nl, plan=plan)
    z = L.ldbp_forward(r, taps, c, ntap, plan=(0, 0, 0, 1))
    unit_diff = float((y - z).abs().max().item())
    ss = nwave * n * ell
    flops = nwave * n * sum(fwd_flops_per_sample_step(t, True) + 4 * kappa + 1 for t in ntap)
    S = 2
    ck = torch.empty((L.num_checkpoints(ell, S),) + tuple(r.shape), dtype=r.dtype, device=dev)
    _, _, gy = TX.rx_mse(z, W["s"], W["p"], RHO_D, RS, want_grad=True)
    bws = torch.empty(E.essm_backward_workspace_size(r, ntap, nl, ckpt=ck, ckpt_every=S), dtype=torch.uint8,
                      device=dev)

    def fwd_bwd():
        E.essm_forward(r, taps, c, eta, ntap, nl, y=y, ckpt=ck, ckpt_every=S, plan=(0, 0, 0, 1), stream=stream)
        E.essm_backward(r, taps, c, eta, ntap, nl, gy, ckpt=ck, ckpt_every=S, need_gx=False, symmetric=True,
                        ws=bws, stream=stream)

    ms_fb = event_time(torch, stream, fwd_bwd, max(5, reps // 5), 2)
    return {"workload": f"64 waveforms x 65,536 c64 samples, l = 50, 15 folded taps, filters of {ne} real taps",
            "kappa": kappa, "plan": list(plan), "passes": npass, "tile_len": tile_len, "steps_per_pass": spp,
            "fwd_ms": ms, "fwd_value": ss / (ms * 1e-3), "unit": "samples*steps/s",
            "fwd_flops_per_sample_step": flops / (nwave * n * ell),
            "fwd_achieved_tflops": flops / (ms * 1e-3) / 1e12,
            "fwd_alu_frac": flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
            "unit_filter_max_abs_diff_vs_ldbp": unit_diff,
            "fwd_bwd_ms": ms_fb, "fwd_bwd_value": ss / (ms_fb * 1e-3), "ckpt_every": S}


def aperiodic_timing(torch, dev, W, plan, reps: int):
    """Overlap-save streaming on the inference workload: the valid edge on 64 blocks of 65,536 output
    samples, each passed with P = sum K samples of context on both sides (the blocks of a continuous
    stream), and the zero edge on the 64 waveforms (zero margins of P)."""
    from paper_2010_14258_amd import aperiodic as A

    r, taps, c, ntap = W["r"], W["taps"], W["c"], W["ntap"]
    nwave, n = r.shape
    ell = len(ntap)
    P = A.halo(ntap)
    stream = torch.cuda.current_stream(dev)
    blocks = torch.cat([r[:, n - P:], r, r[:, :P]], dim=1).contiguous()   # n + 2P input samples per block
    out = {"P": P, "plan": list(plan)}
    for edge, inp in (("valid", blocks), ("zero", r)):
        y = torch.empty_like(r)
        ws = torch.empty(max(A.forward_aperiodic_workspace_size(inp, ntap, edge=edge, plan=plan), 1),
                         dtype=torch.uint8, device=dev)
        ms = event_time(torch, stream, lambda: A.forward_aperiodic(inp, taps, c, ntap, edge, y=y, plan=plan, ws=ws,
                                                                   stream=stream), reps, 2)
        flops = nwave * (n + 2 * P) * sum(fwd_flops_per_sample_step(t, bool(plan[3])) for t in ntap)
        out[edge] = {"ms": ms, "output_samples_steps_per_s": nwave * n * ell / (ms * 1e-3),
                     "processed_samples": nwave * (n + 2 * P), "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                     "alu_frac": flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    out["workload"] = (f"{nwave} blocks of {n} output samples (valid: {n + 2 * P} input samples each; zero: "
                       f"{n} input samples, {n + 2 * P} working samples), l = {ell}, {TAPS} taps")
    return out


def essm_trained(torch, dev, iters: int, powers, kappa: int = 20, ntaps: int = 15, stps: int = 1):
    """Conventional vs generalised ESSM (Sec. III-D, V-C) on the 10 x 100 km link with few steps: l = 10
    (one step per span, log step sizes), least-squares FIR linear steps of `ntaps` taps, filters of
    2 kappa + 1 real taps starting as unit filters.  Conventional: one filter shared by all nonlinear
    steps, the only trained parameters.  Generalised: a filter per step, trained jointly with the
    linear steps and the Kerr coefficients.  LDBP with the same steps and taps (no filters) trained the
    same way, and the least-squares initialisation (= every model before training), for reference.
    Training as the training recipe (32 x 16,384 waveforms per batch, launch powers {2, 3, 4} dBm,
    Adam lr 1e-3), evaluated on the 64 x 65,536 inference batch at each launch power, with FFT-DBP."""
    from paper_2010_14258_amd import essm as E
    from paper_2010_14258_amd import ldbp as L
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import train as TRN
    from paper_2010_14258_amd import txrx as TX

    variants = [("ldbp", dict()),
                ("essm_conventional", dict(essm_kappa=kappa, essm_shared=True, train_taps=False, train_c=False)),
                ("essm_generalised", dict(essm_kappa=kappa))]
    models = []
    init = None
    for name, kw in variants:
        trn = TRN.Trainer(TRN.TrainConfig(iters=iters, t_init=ntaps, t_final=ntaps, ldbp_steps=stps, **kw),
                          device=dev)
        if init is None:
            init = (trn.taps.clone(), trn.c.clone(), list(trn.ntap))
        t0 = time.perf_counter()
        curve = []
        for it in range(iters):
            loss = trn.step(sync=(it + 1) % 250 == 0)
            if (it + 1) % 250 == 0:
                curve.append([it + 1, loss])
                print(f"train {name} {it + 1}/{iters} loss {loss:.4e} {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        m = {"name": name, "train_seconds": time.perf_counter() - t0, "loss_curve": curve,
             "taps": trn.taps.contiguous(), "c": trn.c.contiguous(), "ntap": list(trn.ntap)}
        if trn.essm:
            m["eta"] = trn.eta_per_step().contiguous()
            m["nl_ntap"] = list(trn.nl_ntap)
            m["filters"] = trn.eta.view(-1, 2 * kappa + 1).cpu().numpy().round(5).tolist()
        models.append(m)
        del trn
    rows = []
    for p_dbm in powers:
        W = build_workload(torch, dev, p_dbm=p_dbm)
        r = W["r"]
        row = {"launch_dbm": p_dbm,
               "ls_init_snr_db": snr_db(TX, L.ldbp_forward(r, init[0], init[1], init[2], plan=(0, 0, 0, 1)), W["s"],
                                        W["p"])}
        for m in models:
            if "eta" in m:
                z = E.essm_forward(r, m["taps"], m["c"], m["eta"], m["ntap"], m["nl_ntap"], plan=(0, 0, 0, 1))
            else:
                z = L.ldbp_forward(r, m["taps"], m["c"], m["ntap"], plan=(0, 0, 0, 1))
            row[m["name"] + "_snr_db"] = snr_db(TX, z, W["s"], W["p"])
        row["fft_dbp_snr_db_by_steps_per_span"] = {k: snr_db(TX, SS.fft_dbp(r, W["dbp_link"](k)), W["s"], W["p"])
                                                   for k in (1, 2, 5)}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del W, r
        torch.cuda.empty_cache()
    out_models = [{k: v for k, v in m.items() if k not in ("taps", "c", "ntap", "eta", "nl_ntap")} for m in models]
    return {"workload": f"10 x 100 km, l = {10 * stps} ({stps} step per span), {ntaps} taps, kappa = {kappa}; "
                        "evaluated on 64 waveforms x 65,536 c64 samples",
            "train_iterations": iters, "lr_schedule": lr_schedule, "models": out_models, "by_power": rows}


def e1_reduced(torch, dev, iters: int, powers, out_dir: str, resume=None, stop_at=None, train_c: bool = True,
               lr_schedule: str = "constant", prune_frac=None, rho_a: int = 4, data_pool: int = 0,
               eval_batches: int = 4):
    """The paper's first scenario (Sec. V-A) at reduced training length: 10.7 GBd over 25 x 80 km,
    LDBP on the asymmetric split-step with one step per span (l = 25), symmetric filters pruned from 9
    taps to alternating 5 and 3 taps (overall impulse response 13 * 4 + 12 * 2 + 1 = 77 taps),
    Gaussian symbols, training powers {-2, -1, 0, 1} dBm, Adam lr 1e-3 on the filters and the Kerr
    coefficients (train_c False: fixed nonlinear steps, the paper's setting).  Channel: 50
    uniform steps per span at 4 samples per symbol (the paper simulates at 6) with amplifier noise
    (NF 5 dB).  Effective
    SNR per launch power on held-out batches (4 x 32 x 8,192 symbols) for the trained model, its
    least-squares initialisation, FFT-DBP with 1 and 2 steps per span and linear equalisation.
    resume: a trainer checkpoint of the same configuration to continue from (training resumes bit for
    bit); stop_at: save a checkpoint at that iteration and return without evaluating.
    rho_a: analog oversampling of the simulation (the paper's is 6); data_pool > 0: training cycles
    through that many simulated batches; eval_batches: held-out batches of 32 x 8,192 symbols per power
    (39 give the paper's >= 10^7 symbols per SNR), every method evaluated on the same batches."""
    from paper_2010_14258_amd import train as TRN
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import txrx as TX

    extra = {} if prune_frac is None else {"prune_frac": prune_frac}
    cfg = TRN.TrainConfig(nwave=32, nsym=8192, rho_a=rho_a, rho_d=2, nspan=25, span_km=80.0, channel_steps=50,
                          ldbp_steps=1, t_init=9, t_final=5, t_final_alt=3, iters=iters,
                          powers_dbm=(-2.0, -1.0, 0.0, 1.0), symbols="gauss", seed=1101, train_c=train_c,
                          lr_schedule=lr_schedule, data_pool=data_pool, **extra)
    trn = TRN.Trainer(cfg, device=dev)
    if resume:
        trn.load(resume)
    curve = json.load(open(resume + ".curve.json")) if resume and os.path.exists(resume + ".curve.json") else []
    end = iters if stop_at is None else min(stop_at, iters)
    t0 = time.perf_counter()
    while trn.it < end:
        loss = trn.step(sync=(trn.it + 1) % 500 == 0)
        if trn.it % 500 == 0:
            curve.append([trn.it, loss, int(sum(trn.ntap))])
            print(f"e1 train {trn.it}/{iters} loss {loss:.4e} taps {list(trn.ntap)[:4]}... "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    os.makedirs(out_dir, exist_ok=True)
    ck = os.path.join(out_dir, f"e1_it{trn.it}.pt")
    trn.save(ck)
    json.dump(curve, open(ck + ".curve.json", "w"))
    if trn.it < iters:
        return {"checkpoint": ck, "iteration": trn.it, "train_seconds": train_s}
    init_model = TRN.Trainer(cfg, device=dev)
    links = {"fft_dbp_1stps_snr_db": trn.dbp_link(1), "fft_dbp_2stps_snr_db": trn.dbp_link(2)}
    lin = trn.dbp_link(1)
    lin.gamma = 0.0
    links["linear_eq_snr_db"] = lin
    rows = []
    t_eval = time.perf_counter()
    for p_ in powers:
        err, cnt = {}, 0
        pw = torch.full((cfg.nwave,), 10.0 ** (p_ / 10.0 - 3.0), dtype=torch.float64, device=dev)
        for b in range(eval_batches):
            r, s_, pp = trn.batch(1_000_000 + b, pw)     # the same held-out batch for every method
            outs = {"ldbp_trained_snr_db": trn.forward(r)[0], "ldbp_ls_init_snr_db": init_model.forward(r)[0]}
            for k, lk in links.items():
                outs[k] = SS.fft_dbp(r, lk, npol=cfg.npol)
            for k, z in outs.items():
                mse, _, _ = TX.rx_mse(z, s_, pp, cfg.rho_d, cfg.rs, cfg.rolloff, npol=cfg.npol)
                err[k] = err.get(k, 0.0) + float(mse.sum().item())
            cnt += cfg.nwave
        row = {"launch_dbm": p_, "symbols": cnt * cfg.nsym}
        row.update({k: 10.0 * math.log10(cnt / v) for k, v in err.items()})
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    eval_s = time.perf_counter() - t_eval
    del init_model
    resp = 1 + sum(t - 1 for t in trn.ntap)
    peak = {k: max(r[k] for r in rows) for k in rows[0] if k.endswith("_snr_db")}
    return {"workload": "10.7 GBd, 25 x 80 km SSMF, Gaussian symbols, LDBP l = 25 (1 step per span), 9 -> 5/3 taps",
            "train_kerr_coefficients": train_c, "lr_schedule": lr_schedule, "prune_frac": cfg.prune_frac,
            "analog_oversampling": rho_a, "data_pool": data_pool, "eval_batches_per_power": eval_batches,
            "eval_seconds": eval_s,
            "train_iterations": iters, "train_seconds_last_call": train_s, "final_ntap": list(trn.ntap),
            "impulse_response_taps": resp, "loss_curve": curve, "by_power": rows, "peak_snr_db": peak,
            "paper_context": {"ldbp_peak_snr_db": 23.5, "penalty_vs_fd_dbp_1stps_db": 2.0,
                              "train_iterations": 150000, "analog_oversampling": 6,
                              "note": "the paper's values (Sec. V-A, Fig. results_Ip2008), context only"}}


def e8_reduced(torch, dev, iters: int, powers, rho_a: int = 4, data_pool: int = 0, eval_batches: int = 4,
               lr_schedule: str = "constant"):
    """The paper's 32 GBd scenario (Sec. V-F): 10 x 100 km, LDBP on the symmetric split-step with log
    step sizes, 2 steps per span (l = 21, 23 taps per filter: an overall impulse response of
    21 * 22 + 1 = 463 taps) trained at P = {3, 4, 5} dBm, and 4 steps per span (l = 41, 13 taps: 493)
    at {4, 5, 6} dBm; Gaussian symbols, no pruning, Adam lr 1e-3 on the filters and the Kerr
    coefficients (the last step stays linear).  Channel at rho_a samples per symbol (the paper: 6) with
    100 steps per span and amplifier noise; data_pool > 0: training cycles through that many simulated
    batches.  Effective SNR per power on eval_batches held-out batches of 32 x 8,192 symbols, with
    FFT-DBP at the same number of steps per span (and 10) for reference, on the same waveforms.
    lr_schedule "cosine": Adam's step size decays from 1e-3 to 1e-4 by a half cosine over the run."""
    from paper_2010_14258_amd import train as TRN

    out = {}
    for stps, ntaps, ptrain in ((2, 23, (3.0, 4.0, 5.0)), (4, 13, (4.0, 5.0, 6.0))):
        cfg = TRN.TrainConfig(nwave=32, nsym=8192, rho_a=rho_a, rho_d=2, rs=32e9, nspan=10, span_km=100.0,
                              channel_steps=100, ldbp_steps=stps, t_init=ntaps, t_final=ntaps, iters=iters,
                              powers_dbm=ptrain, symbols="gauss", ssm="symmetric", seed=1301 + stps,
                              data_pool=data_pool, lr_schedule=lr_schedule)
        trn = TRN.Trainer(cfg, device=dev)
        nb = eval_batches
        init = {p_: trn.evaluate(nbatch=nb, p_dbm=p_) for p_ in powers}
        t0 = time.perf_counter()
        curve = []
        while trn.it < iters:
            every = 500 if iters <= 20000 else 5000
            loss = trn.step(sync=(trn.it + 1) % every == 0)
            if trn.it % every == 0:
                curve.append([trn.it, loss])
                print(f"e8 {stps} StPS {trn.it}/{iters} loss {loss:.4e} {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        train_s = time.perf_counter() - t0
        rows = []
        for p_ in powers:
            row = {"launch_dbm": p_, "ldbp_trained_snr_db": trn.evaluate(nbatch=nb, p_dbm=p_),
                   "ldbp_ls_init_snr_db": init[p_],
                   "fft_dbp_same_stps_snr_db": trn.evaluate_fft_dbp(stps, nbatch=nb, p_dbm=p_),
                   "fft_dbp_10stps_snr_db": trn.evaluate_fft_dbp(10, nbatch=nb, p_dbm=p_)}
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
        peak = {k: max(r[k] for r in rows) for k in rows[0] if k.endswith("_snr_db")}
        out[f"{stps}_stps"] = {"l": len(trn.ntap), "taps_per_filter": ntaps,
                               "impulse_response_taps": 1 + sum(t - 1 for t in trn.ntap),
                               "train_powers_dbm": list(ptrain), "train_seconds": train_s, "loss_curve": curve,
                               "by_power": rows, "peak_snr_db": peak,
                               "peak_gain_over_fft_dbp_same_stps_db": peak["ldbp_trained_snr_db"]
                               - peak["fft_dbp_same_stps_snr_db"]}
        del trn
    return {"workload": "32 GBd, 10 x 100 km SSMF, Gaussian symbols, symmetric-SSM LDBP, 2 and 4 steps per span",
            "train_iterations": iters, "rho_a": rho_a, "data_pool": data_pool,
            "symbols_per_snr": eval_batches * 32 * 8192, "lr_schedule": lr_schedule, "models": out,
            "paper_context": {"gain_over_dbp_db": {"2_stps": 2.1, "4_stps": 0.6}, "taps": 463,
                              "note": "the paper's values (Sec. V-F), after 150,000 + 1,500 iterations; context only"}}


def init_schemes(torch, dev, iters: int, every: int = 1000, schemes=("least_squares", "unit", "random"),
                 ntaps: int = 9):
    """Initialisation study (Sec. V-E) on the 25 x 80 km link: LDBP with one step per span and 9 general
    (unconstrained) taps per step, no pruning, trained at P = {0 dBm} with Gaussian symbols from
    least-squares, unit and random filters (random: i.i.d. N(0, 1) parts divided by the sum of squared
    magnitudes; multiobjective: the least-squares filters refined jointly by the multi-objective
    weighted least squares of Sec. VI-B).  Learning curves: effective SNR at 0 dBm on held-out batches
    every `every` iterations."""
    from paper_2010_14258_amd import train as TRN

    out = {}
    options = {"least_squares": {}, "unit": {"unit_init": True}, "random": {"random_init": True},
               "multiobjective": {"init_method": "multiobjective"}}
    for name in schemes:
        kw = options[name]
        cfg = TRN.TrainConfig(nwave=32, nsym=8192, rho_a=4, rho_d=2, nspan=25, span_km=80.0, channel_steps=50,
                              ldbp_steps=1, t_init=ntaps, t_final=ntaps, iters=iters, powers_dbm=(0.0,),
                              symbols="gauss", symmetric=False, seed=1201, **kw)
        trn = TRN.Trainer(cfg, device=dev)
        curve = [[0, trn.evaluate(nbatch=2, p_dbm=0.0)]]
        t0 = time.perf_counter()
        while trn.it < iters:
            trn.step(sync=False)
            if trn.it % every == 0:
                curve.append([trn.it, trn.evaluate(nbatch=2, p_dbm=0.0)])
                print(f"init {name} {trn.it}/{iters} SNR {curve[-1][1]:.2f} dB {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        out[name] = {"snr_curve_db": curve, "final_snr_db": trn.evaluate(nbatch=4, p_dbm=0.0),
                     "train_seconds": time.perf_counter() - t0}
        del trn
    return {"workload": f"10.7 GBd, 25 x 80 km, Gaussian symbols, LDBP l = 25, {ntaps} taps, trained at 0 dBm",
            "train_iterations": iters, "schemes": out,
            "paper_context": {"least_squares_db": 25.6, "unit_db": 25.1, "random": "stuck", "iterations": 10000,
                              "note": "the paper's values (Sec. V-E, Fig. results(c)), context only"}}


COPY_PROBE_ELEMS = 64 << 20   # complex64 elements: 512 MiB per buffer, beyond the last-level cache


def copy_probe(torch, dev):
    """Three device-to-device copies of 512 MiB: a plain kernel of known traffic, against which the
    FETCH_SIZE and WRITE_SIZE counters of the same run are calibrated."""
    big = torch.empty(COPY_PROBE_ELEMS, dtype=torch.complex64, device=dev)
    dst = torch.empty_like(big)
    for _ in range(3):
        dst.copy_(big)
    torch.cuda.synchronize()


def streaming_probe(torch, dev, reps: int):
    """What plain streaming kernels reach on this GPU (512 MiB in, 512 MiB out, beyond the last-level
    cache): a device-to-device copy and an elementwise scaling, HIP-event timed; read + write bytes."""
    x = torch.ones(COPY_PROBE_ELEMS, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    moved = 2 * COPY_PROBE_ELEMS * 8
    ms_copy = event_time(torch, stream, lambda: y.copy_(x), reps, 2)
    ms_scale = event_time(torch, stream, lambda: torch.mul(x, 2.0, out=y), reps, 2)
    return {"bytes_moved": moved, "copy_ms": ms_copy, "copy_gbs": moved / (ms_copy * 1e-3) / 1e9,
            "scale_ms": ms_scale, "scale_gbs": moved / (ms_scale * 1e-3) / 1e9}


def pick_dbp_setting(sweep, snr_ldbp: float):
    """FFT-DBP setting to compare with: the fewest steps per span whose SNR is within 0.1 dB of LDBP's
    (equal SNR).  When no setting reaches LDBP, the fewest steps per span within 0.1 dB of the best
    FFT-DBP SNR, flagged as not at equal SNR.  Returns (steps per span, at_equal_snr)."""
    keys = sorted(sweep)
    for k in keys:
        if sweep[k] >= snr_ldbp - 0.1:
            return k, True
    best = max(sweep.values())
    return next(k for k in keys if sweep[k] >= best - 0.1), False


def snr_db(TX, z, s, p):
    mse, _, _ = TX.rx_mse(z, s, p, RHO_D, RS)
    return 10.0 * math.log10(1.0 / float(mse.mean().item()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-waves", type=int, default=48, help="waveforms in the oracle's bounded sample")
    ap.add_argument("--mode", choices=["full", "fwd", "pmc", "bwd", "train", "variants", "dbp", "snr", "essm", "e1",
                                       "init", "e8", "roof", "manakov", "manakov_train", "uneven_snr", "fft_lengths"],
                    default="full",
                    help="fwd: forward timing only (for kernel traces); pmc: a few forwards and a copy probe; "
                         "bwd: the training step (checkpointed forward + backward) and a copy probe; "
                         "train: whole training iterations (channel simulation to Adam) for kernel traces; "
                         "variants: the generalised ESSM and overlap-save timings alone (fixed plans); "
                         "dbp: FFT-DBP at one step per span only (for kernel traces of the split-step passes); "
                         "snr: train LDBP, then the equal-SNR comparison with FFT-DBP over launch powers; "
                         "essm: train conventional and generalised ESSM (and LDBP) with one step per span; "
                         "e1: the 25 x 80 km scenario with Gaussian symbols and 9 -> 5/3-tap pruning; "
                         "init: least-squares, unit and random initialisation on that link; "
                         "e8: the 32 GBd scenario (symmetric-SSM LDBP, 2 and 4 steps per span); "
                         "roof: the 1,024-waveform forward at 1-10 steps per pass (where the memory roof sits); "
                         "manakov: dual-polarisation forward and forward + backward on 8 x 2^20 x 2 and a copy "
                         "probe (for kernel traces and counters); "
                         "manakov_train: train the dual-polarisation 8 x 2^20 x 2 configuration (--train-iters, "
                         "--powers); uneven_snr: the uneven serving batch on simulated inputs, trained span models, "
                         "LDBP against FFT-DBP at 1-10 steps per span (--train-iters per tap count); "
                         "fft_lengths: FFT-DBP step time at power-of-two and 5-smooth lengths")
    ap.add_argument("--train-iters", type=int, default=5000, help="training iterations of --mode snr")
    ap.add_argument("--powers", default="-4,-2,0,1,2,3,4,5,6", help="launch powers (dBm) of --mode snr")
    ap.add_argument("--resume", default=None, help="--mode e1: trainer checkpoint to continue from")
    ap.add_argument("--fixed-c", action="store_true", help="--mode e1: keep the Kerr coefficients fixed")
    ap.add_argument("--prune-frac", type=float, default=None,
                    help="--mode e1: fraction of the iterations over which the pruning events fall "
                         "(default: the trainer's)")
    ap.add_argument("--rho-a", type=int, default=4, help="--mode e1: analog oversampling of the simulation")
    ap.add_argument("--eval-batches", type=int, default=4,
                    help="--mode e1: held-out batches of 32 x 8,192 symbols per launch power")
    ap.add_argument("--lr-schedule", default="constant", choices=["constant", "cosine"],
                    help="--mode e1, e8 and snr: Adam step size; cosine: decay to 1e-4 after the last pruning event")
    ap.add_argument("--stop-at", type=int, default=None, help="--mode e1: checkpoint at this iteration and stop")
    ap.add_argument("--out-dir", default=None,
                    help="--mode e1: directory of the trainer checkpoints and learning curve (default: the "
                         "system temporary directory)")
    ap.add_argument("--schemes", default="least_squares,unit,random",
                    help="--mode init: initialisations (least_squares, unit, random, multiobjective)")
    ap.add_argument("--init-taps", type=int, default=9, help="--mode init: taps per step")
    ap.add_argument("--data-pool", type=int, default=0,
                    help="--mode snr: training batches cycle through this many fixed batches (0: fresh batches)")
    ap.add_argument("--train-taps", default="25:3",
                    help="models of --mode snr: initial:final taps per step, comma separated (pruned in training)")
    ap.add_argument("--one-stream", action="store_true",
                    help="fwd/pmc/bwd modes: keep every launch on one stream (the kernel's own per-launch time)")
    ap.add_argument("--plan", default=None,
                    help="forward plan S,chunks,outputs_per_thread,symmetric[,one_stream] (default: the fixed "
                         "headline plan 10,1,7,1)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the forward autotuner's plans instead of the fixed ones")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline and args.mode == "full":
        cpu = cpu_baseline(args.cpu_waves, RHO_D * NSYM, [TAPS] * (NSPAN * LDBP_STPS))

    import torch
    from paper_2010_14258_amd import _native
    from paper_2010_14258_amd import ldbp as L
    from paper_2010_14258_amd import ssm as SS
    from paper_2010_14258_amd import txrx as TX

    _native.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.mode == "train":
        # training iterations alone on the 32 x 16,384 configuration (l = 50, 25 -> 3 taps, channel
        # 1,000 steps): transmitter, channel, receiver, LDBP forward and backward, loss, Adam
        from paper_2010_14258_amd import train as TRN
        trn = TRN.Trainer(TRN.TrainConfig(iters=5000), device=dev)
        for _ in range(max(1, args.warmup)):
            trn.step(sync=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            trn.step(sync=False)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "train", "iteration_ms": (time.perf_counter() - t1) / args.steps * 1e3,
                          "iterations": args.steps, "warmup": max(1, args.warmup)}), flush=True)
        return
    W = build_workload(torch, dev, cheap=args.mode != "full")
    r, taps, c, ntap = W["r"], W["taps"], W["c"], W["ntap"]
    nwave, n = r.shape
    ell = len(ntap)
    y = torch.empty_like(r)
    if args.mode == "snr":
        variants = [tuple(int(t) for t in v.split(":")) for v in args.train_taps.split(",")]
        out = equal_snr_trained(torch, dev, args.train_iters, [float(v) for v in args.powers.split(",")], 20,
                                variants, args.data_pool, args.lr_schedule)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "e1":
        out = e1_reduced(torch, dev, args.train_iters, [float(v) for v in args.powers.split(",")],
                         args.out_dir or tempfile.gettempdir(), args.resume, args.stop_at, not args.fixed_c,
                         args.lr_schedule, args.prune_frac, args.rho_a, args.data_pool, args.eval_batches)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "fft_lengths":
        print(json.dumps(fft_lengths(torch, dev, args.steps)), flush=True)
        return
    if args.mode == "uneven_snr":
        print(json.dumps(uneven_serving(torch, dev, args.steps, args.train_iters)), flush=True)
        return
    if args.mode == "manakov_train":
        print(json.dumps(manakov_trained(torch, dev, args.train_iters,
                                         [float(v) for v in args.powers.split(",")])), flush=True)
        return
    if args.mode == "e8":
        print(json.dumps(e8_reduced(torch, dev, args.train_iters, [float(v) for v in args.powers.split(",")],
                                    args.rho_a, args.data_pool, args.eval_batches, args.lr_schedule)), flush=True)
        return
    if args.mode == "init":
        print(json.dumps(init_schemes(torch, dev, args.train_iters, schemes=args.schemes.split(","),
                                      ntaps=args.init_taps)), flush=True)
        return
    if args.mode == "essm":
        out = essm_trained(torch, dev, args.train_iters, [float(v) for v in args.powers.split(",")])
        print(json.dumps(out), flush=True)
        return
    if args.mode == "dbp":
        # FFT-DBP at one step per span on the same received batch (the split-step passes alone)
        link = W["dbp_link"](1)
        wsd = torch.empty(SS.ssm_workspace_size(r, link), dtype=torch.uint8, device=dev)
        ms = event_time(torch, stream, lambda: SS.fft_dbp(r, link, y=y, ws=wsd, stream=stream), args.steps,
                        args.warmup)
        nstep = link.nspan * link.nstep
        print(json.dumps({"fft_dbp_ms": ms, "dbp_steps": nstep, "us_per_step": ms / nstep * 1e3,
                          "nwave": nwave, "n": n}))
        return
    if args.mode == "bwd":
        # the training step alone: forward with 2-step block checkpoints + backward (folded symmetric
        # filters, the gradient reduction included), then the copy probe that calibrates the counters
        S = 2
        ck = torch.empty((L.num_checkpoints(ell, S),) + tuple(r.shape), dtype=r.dtype, device=dev)
        z = L.ldbp_forward(r, taps, c, ntap)
        _, _, gy = TX.rx_mse(z, W["s"], W["p"], RHO_D, RS, want_grad=True)
        bws = torch.empty(L.ldbp_backward_workspace_size(r, ntap, ckpt=ck, ckpt_every=S), dtype=torch.uint8,
                          device=dev)

        fplan = (0, 0, 0, 1, 1) if args.one_stream else (0, 0, 0, 1)

        def fwd_bwd():
            L.ldbp_forward(r, taps, c, ntap, y=y, ckpt=ck, ckpt_every=S, plan=fplan, stream=stream)
            L.ldbp_backward(r, taps, c, ntap, gy, ckpt=ck, ckpt_every=S, need_gx=False, symmetric=True,
                            ws=bws, stream=stream, one_stream=args.one_stream)

        ms = event_time(torch, stream, fwd_bwd, args.steps, args.warmup)
        copy_probe(torch, dev)
        print(json.dumps({"mode": "bwd", "fwd_bwd_ms": ms, "ckpt_every": S, "one_stream": args.one_stream,
                          "nwave": nwave, "n": n, "steps_l": ell, "taps": TAPS,
                          "copy_probe": "3 copies of 512 MiB"}), flush=True)
        return
    if args.mode == "manakov":
        out = manakov(torch, dev, max(3, args.steps))
        copy_probe(torch, dev)
        out["mode"] = "manakov"
        out["copy_probe"] = "3 copies of 512 MiB"
        print(json.dumps(out), flush=True)
        return
    if args.mode == "roof":
        # where the memory roof sits: the forward on 1,024 waveforms (512 MiB per buffer, beyond the
        # last-level cache) at 1 to 10 steps per pass, every launch on one stream, then the copy probe
        # that calibrates FETCH_SIZE / WRITE_SIZE in counter runs
        out = {"mode": "roof", "plans": roof_sweep(torch, dev, W, args.steps, args.warmup),
               "streaming": streaming_probe(torch, dev, args.steps)}
        copy_probe(torch, dev)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "variants":
        # the generalised ESSM (forward; forward with checkpoints + backward) and overlap-save streaming
        # alone, with fixed plans, for kernel traces; first bring the GPU to its steady clock
        for _ in range(600):
            L.ldbp_forward(r, taps, c, ntap, y=y, plan=(10, 1, 7, 1), stream=stream)
        torch.cuda.synchronize()
        out = {"mode": "variants", "essm": essm_timing(torch, dev, W, args.steps, plan=(3, 1, 7, 1)),
               "aperiodic": aperiodic_timing(torch, dev, W, (10, 1, 7, 1), args.steps)}
        print(json.dumps(out), flush=True)
        return
    from paper_2010_14258_amd import autotune as AT
    plan_gen = GENERAL_PLAN
    if args.plan:
        plan = tuple(int(v) for v in args.plan.split(","))
    elif args.autotune:
        plan, _, _ = AT.tune_forward(r, taps, c, ntap, symmetric=True, reps=10)
        plan_gen, _, _ = AT.tune_forward(r, taps, c, ntap, symmetric=False, reps=10)
    else:
        plan = HEADLINE_PLAN
    if args.mode != "pmc":
        # bring the GPU to its steady clock before anything is timed (about 0.2 s of work)
        for _ in range(600):
            L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan, stream=stream)
        torch.cuda.synchronize()
    folded = bool(plan[3])
    ws = torch.empty(max(L.ldbp_forward_workspace_size(r, ntap, plan=plan), 1), dtype=torch.uint8, device=dev)

    plan1 = tuple(plan[:4]) + (1,)   # the same plan with every launch on the caller's stream

    def fwd():
        L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan1 if args.one_stream else plan, ws=ws, stream=stream)

    def fwd_one():
        L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan1, ws=ws, stream=stream)

    if args.mode == "pmc":
        for _ in range(3):
            fwd()
        copy_probe(torch, dev)
        print(json.dumps({"pmc_probe": True, "plan": list(plan),
                          "fwd_launches": 3 * L.ldbp_forward_plan_query(0, 1, nwave, n, ntap, plan=plan)[0],
                          "copy_bytes": 2 * COPY_PROBE_ELEMS * 8, "kernel_hash": kernel_hash()}))
        return

    t0 = time.perf_counter()
    ms_fwd = event_time(torch, stream, fwd, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    dist = time_distribution(torch, stream, fwd, args.steps, 2)
    npass, tile_len, spp = L.ldbp_forward_plan_query(0, 1, nwave, n, ntap, plan=plan)
    ss = nwave * n * ell
    value = ss / (ms_fwd * 1e-3)
    # the kernel's own per-launch time: the same plan with every launch on the caller's stream (the
    # default call runs the two halves of the batch on two streams, whose launches overlap)
    ms_one = event_time(torch, stream, fwd_one, args.steps, args.warmup)
    launch_ms = ms_one / npass
    flops_fwd = nwave * n * sum(fwd_flops_per_sample_step(t, folded) for t in ntap)
    flops_launch = flops_fwd / npass
    achieved_tflops = flops_launch / (launch_ms * 1e-3) / 1e12
    bytes_launch = nwave * n * 8 * 2
    achieved_gbs = bytes_launch / (launch_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        # counter runs of this kernel source, one entry per plan the autotuner has picked
        with open(TRAFFIC_FILE) as fh:
            entries = json.load(fh).get("entries", [])
        for tr in entries:
            if tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == [nwave, n, ell, TAPS] \
                    and tr.get("plan") == list(plan):
                traffic = tr.get("bytes_per_launch")

    out = {
        "metric": "samples*steps/s of the LDBP forward (waveform samples x LDBP steps per second)",
        "value": value,
        "unit": "samples*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fwd,
        "wall_s": wall,
        "per_call": dist,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic: GPU-simulated 16-QAM over 10 x 100 km SSMF with ASE (library kernels)",
        "config": {"workload": "LDBP inference, 64 waveforms x 65,536 c64 samples, l = 50 (5 steps/span), 15 taps",
                   "nwave": nwave, "n": n, "steps_l": ell, "taps": TAPS, "launch_dbm": P_DBM,
                   "plan": list(plan), "folded_symmetric_filters": folded,
                   "passes": npass, "tile_len": tile_len, "steps_per_pass": spp},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": f"ldbp_fwd_kernel<float,1,{plan[2]},256>" + (" folded" if folded else ""),
                     "launch_ms": launch_ms, "one_stream_ms_per_step": ms_one,
                     "flops_per_launch": flops_launch, "algorithmic_bytes_per_launch": bytes_launch,
                     "hbm_achieved_gbs": achieved_gbs, "hbm_frac": achieved_gbs / HBM_PEAK_GBS,
                     "split_batch_achieved": flops_fwd / (ms_fwd * 1e-3) / 1e12,
                     "split_batch_frac": flops_fwd / (ms_fwd * 1e-3) / 1e12 / FP32_PEAK_TFLOPS},
    }

    if args.mode == "full":
        ms_gen_tuned = event_time(torch, stream, lambda: L.ldbp_forward(r, taps, c, ntap, y=y, plan=plan_gen,
                                                                         stream=stream), args.steps, 2)
        fl_gen = nwave * n * sum(fwd_flops_per_sample_step(t) for t in ntap)
        out["general_taps_forward"] = {"value": ss / (ms_gen_tuned * 1e-3), "unit": "samples*steps/s",
                                       "ms_per_step": ms_gen_tuned, "plan": list(plan_gen),
                                       "achieved_tflops": fl_gen / (ms_gen_tuned * 1e-3) / 1e12,
                                       "frac": fl_gen / (ms_gen_tuned * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    if args.mode == "full":
        # forward with block checkpoints + backward
        S = 2
        ck = torch.empty((L.num_checkpoints(ell, S),) + tuple(r.shape), dtype=r.dtype, device=dev)
        z = L.ldbp_forward(r, taps, c, ntap)
        _, _, gy = TX.rx_mse(z, W["s"], W["p"], RHO_D, RS, want_grad=True)
        bws = torch.empty(L.ldbp_backward_workspace_size(r, ntap, ckpt=ck, ckpt_every=S), dtype=torch.uint8,
                          device=dev)

        def fwd_bwd(sym):
            L.ldbp_forward(r, taps, c, ntap, y=y, ckpt=ck, ckpt_every=S, plan=(0, 0, 0, sym), stream=stream)
            L.ldbp_backward(r, taps, c, ntap, gy, ckpt=ck, ckpt_every=S, need_gx=False, symmetric=bool(sym),
                            ws=bws, stream=stream)

        ms_fb = event_time(torch, stream, lambda: fwd_bwd(1), max(5, args.steps // 5), 2)
        ms_fb_gen = event_time(torch, stream, lambda: fwd_bwd(0), max(5, args.steps // 5), 2)
        # the backward kernel's own position: the backward call alone with every launch on one stream,
        # one launch per block of S steps over the whole batch (the two small gradient-reduction
        # launches, about 1% of the call, are included in the per-launch time)
        ms_b = event_time(torch, stream,
                          lambda: L.ldbp_backward(r, taps, c, ntap, gy, ckpt=ck, ckpt_every=S, need_gx=False,
                                                  symmetric=True, ws=bws, stream=stream, one_stream=True),
                          max(5, args.steps // 5), 2)
        nblk = -(-ell // S)
        b_launch_ms = ms_b / nblk
        # every block but the last reads its output (the next block's checkpoint) instead of recomputing
        # its last step, so the algorithmic work leaves that step's forward arithmetic out
        skipped = sum(fwd_flops_per_sample_step(ntap[min(ell, (j + 1) * S) - 1], True) for j in range(nblk - 1))
        b_flops_launch = nwave * n * (sum(bwd_flops_per_sample_step(t, True) for t in ntap) - skipped) / nblk
        b_tflops = b_flops_launch / (b_launch_ms * 1e-3) / 1e12
        # read the block checkpoint, G_y and (not for the last block) the block's output, write G_x (not
        # for the first block: need_gx=False)
        b_bytes_launch = nwave * n * 8 * (2 * nblk + 2 * (nblk - 1)) / nblk
        b_traffic = None
        if os.path.exists(BWD_TRAFFIC_FILE):
            with open(BWD_TRAFFIC_FILE) as fh:
                tr = json.load(fh)
            if tr.get("kernel_hash") == kernel_hash(BWD_KERNEL_SOURCES) \
                    and tr.get("workload") == [nwave, n, ell, TAPS, S]:
                b_traffic = tr.get("bytes_per_launch")
        out["fwd_bwd"] = {"value": ss / (ms_fb * 1e-3), "unit": "samples*steps/s", "ms_per_step": ms_fb,
                          "ckpt_every": S, "folded_symmetric_filters": True,
                          "general_taps_ms": ms_fb_gen, "general_taps_value": ss / (ms_fb_gen * 1e-3),
                          "backward_roofline": {
                              "bound": "alu", "achieved": b_tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": b_tflops / FP32_PEAK_TFLOPS, "traffic": b_traffic,
                              "kernel": "ldbp_bwd_kernel<float,1,5,5,256,false,7> folded", "launch_ms": b_launch_ms,
                              "launches": nblk, "one_stream_backward_ms": ms_b,
                              "flops_per_sample_step": b_flops_launch * nblk / (nwave * n * ell),
                              "flops_per_launch": b_flops_launch, "algorithmic_bytes_per_launch": b_bytes_launch,
                              "hbm_achieved_gbs": b_bytes_launch / (b_launch_ms * 1e-3) / 1e9,
                              "note": "every block but the last reads its output from the next checkpoint, so the "
                                      "algorithmic flops count one recomputed step per block (%d flops per "
                                      "sample*step with both)" % bwd_flops_per_sample_step(TAPS, True)}}
        # equal-SNR comparison with FFT-DBP on the same waveforms
        snr_ldbp = snr_db(TX, z, W["s"], W["p"])
        sweep = {}
        for k in (1, 2, 3, 5, 10, 20):
            link = W["dbp_link"](k)
            zd = SS.fft_dbp(r, link)
            sweep[k] = snr_db(TX, zd, W["s"], W["p"])
        k, equal = pick_dbp_setting(sweep, snr_ldbp)
        link = W["dbp_link"](k)
        yd = torch.empty_like(r)
        dws = torch.empty(SS.ssm_workspace_size(r, link), dtype=torch.uint8, device=dev)
        ms_dbp = event_time(torch, stream, lambda: SS.fft_dbp(r, link, y=yd, ws=dws, stream=stream),
                            max(3, args.steps // 10), 1)
        link1 = W["dbp_link"](1)
        ms_dbp1 = event_time(torch, stream, lambda: SS.fft_dbp(r, link1, y=yd, ws=dws, stream=stream),
                             max(3, args.steps // 10), 1)
        out["equal_snr"] = {
            "ldbp_snr_db": snr_ldbp, "fft_dbp_snr_db_by_steps_per_span": sweep,
            "fft_dbp_steps_per_span": k, "fft_dbp_reaches_ldbp_snr": equal,
            "ldbp_equalised_samples_per_s": nwave * n / (ms_fwd * 1e-3),
            "fft_dbp_equalised_samples_per_s": nwave * n / (ms_dbp * 1e-3),
            ("ldbp_speedup_at_equal_snr" if equal else "ldbp_speedup_vs_best_fft_dbp_unequal_snr"): ms_dbp / ms_fwd,
            "fft_dbp_1stps_samples_steps_per_s": nwave * n * NSPAN / (ms_dbp1 * 1e-3),
            "fft_dbp_1stps_ms": ms_dbp1,
        }
        # one iteration of the 32 x 16,384 training configuration (l = 50, 25 taps, channel 1,000 steps)
        from paper_2010_14258_amd import train as TRN
        trn = TRN.Trainer(TRN.TrainConfig(iters=5000), device=dev)
        trn.step(sync=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            trn.step(sync=False)
        torch.cuda.synchronize()
        out["train_iteration_ms"] = (time.perf_counter() - t1) / 3 * 1e3
        del trn
        out["uneven_batch"] = uneven_batch(torch, dev, max(5, args.steps // 5))
        out["big_batch"] = big_batch(torch, dev, W, max(5, args.steps // 5))
        out["manakov"] = manakov(torch, dev, max(5, args.steps // 5))
        out["essm"] = essm_timing(torch, dev, W, args.steps)
        out["aperiodic"] = aperiodic_timing(torch, dev, W, plan, max(5, args.steps // 2))

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def _oracle_ldbp_chunk(args):
    """One worker's share of the oracle baseline: LDBP forward on `k` seeded waveforms."""
    import synth
    from oracle import ldbp as O

    seed, k, n, ntap = args
    taps = synth.random_taps(1, ntap)
    c = np.full(len(ntap), -1e-2)
    x = synth.complex_normal(seed, (k, n)) * 0.05
    O.ldbp_forward(x, taps, c)
    return k


def cpu_baseline(nw, n, ntap):
    """The FP64 oracle (plain NumPy, not tuned) on the host, on a bounded sample of the same workload
    shape: LDBP by direct convolution in one process (NumPy runs these element-wise operations on one
    core) and over a fork pool of one process per core of the CPU set (at most 16); FFT-DBP at one step
    per span in one process.  Runs before the GPU is touched."""
    import multiprocessing as mp
    import platform

    import synth
    from oracle import ssm as OS

    ell = len(ntap)
    t0 = time.perf_counter()
    _oracle_ldbp_chunk((2, nw, n, ntap))
    dt1 = time.perf_counter() - t0
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    per = 4
    jobs = [(100 + j, per, n, ntap) for j in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_ldbp_chunk, [(99, 1, 256, ntap)] * cores)   # start the workers
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_ldbp_chunk, jobs))
        dtp = time.perf_counter() - t0
    # FFT-DBP, 1 step per span over 10 x 100 km
    alpha = 0.2 * math.log(10) / 10 / 1e3
    link = OS.Link(fs=RHO_D * RS, alpha=alpha, beta2=-21.683e-27, gamma=1.3e-3, span_len=SPAN_KM * 1e3,
                   nspan=NSPAN, step_len=[SPAN_KM * 1e3])
    nd = 16
    r = synth.complex_normal(3, (nd, n)) * 0.05
    t0 = time.perf_counter()
    OS.fft_dbp(r, link)
    dtd = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": done * n * ell / dtp, "unit": "samples*steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} waveforms x {n} samples x {ell} steps ({ntap[0]} taps), FP64 NumPy direct convolution "
                      f"over a pool of {cores} processes, {dtp:.1f} s",
            "single_core": {"value": nw * n * ell / dt1, "cores": 1,
                            "sample": f"{nw} waveforms in one process, {dt1:.1f} s"},
            "fft_dbp_single_core": {"value": nd * n * NSPAN / dtd, "unit": "samples*steps/s", "cores": 1,
                                    "sample": f"{nd} waveforms, FFT-DBP 1 step/span x {NSPAN} spans, NumPy FFT, "
                                              f"{dtd:.1f} s"},
            "host": {"cpu_model": model, "os_cpu_count": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0)), "python": platform.python_version()},
            "note": "the FP64 correctness oracle timed as it stands, not a tuned CPU implementation"}


if __name__ == "__main__":
    main()
