"""Pins for the parameter-initialisation oracle (Sec. IV-C) and the printed arithmetic (Sec. V)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import design as D
from oracle import ldbp as L
from oracle import ssm as S
from oracle import train as TR
from oracle import units as U

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
ALPHA = U.alpha_from_db_per_km(0.2)
BETA2 = U.beta2_from_ps2_per_km(-21.683)
GAMMA = U.gamma_from_per_w_per_km(1.3)


def test_example1_step_sizes_and_merge():
    g = GOLD["example1"]
    span = g["span_km"] * 1e3
    steps = D.log_steps(span, g["steps_per_span"], ALPHA)
    plan = D.dbp_step_plan(span, g["nspan"], steps)
    deltas = [d / 1e3 for d, _ in plan]
    np.testing.assert_allclose(deltas, g["deltas_dbp_order_km"], atol=g["tolerance_km"])
    merged = [m / 1e3 for m in D.merge_half_steps([d for d, _ in plan])]
    np.testing.assert_allclose(merged, g["merged_km"], atol=g["tolerance_km"])
    taps, c = D.init_symmetric(span, g["nspan"], steps, 15, 21.4e9, ALPHA, BETA2, GAMMA)
    ids = [i - 1 for i in g["identical_filters_1based"]]
    for i in ids[1:]:
        np.testing.assert_allclose(taps[i], taps[ids[0]], atol=1e-13)
    assert np.max(np.abs(taps[0] - taps[ids[0]])) > 1e-3
    assert c[-1] == 0.0 and len(taps) == 5


def test_least_squares_on_dft_grid_is_truncated_idft():
    # On the N-point grid the columns of B are orthogonal (Parseval), so LS = truncated inverse DFT.
    N, T, xi = 512, 15, 0.5
    K = (T - 1) // 2
    w = 2 * np.pi * np.arange(-N // 2, N // 2) / N
    B = np.exp(-1j * np.outer(w, np.arange(-K, K + 1)))
    h_ls, *_ = np.linalg.lstsq(B, np.exp(1j * xi * w * w), rcond=None)
    np.testing.assert_allclose(D.truncated_idft_taps(xi, T, N), h_ls, atol=1e-13)
    # The paper's (N+1)-point grid converges to it as N grows.
    assert np.max(np.abs(D.ls_taps(xi, T, 8192) - D.truncated_idft_taps(xi, T, 8192))) < 1e-3


def test_ls_taps_symmetric():
    h = D.ls_taps(0.8, 11, 2048)
    np.testing.assert_allclose(h, h[::-1], atol=1e-12)


def test_initialised_full_length_ldbp_equals_fft_dbp():
    # With T = n (odd) and unit-gain inverse-CD taps, the DBP-initialised LDBP is exactly FFT-DBP (Sec. III-B, IV-C).
    n = 129
    fs = 21.4e9
    steps = D.log_steps(100e3, 3, ALPHA)
    link = S.Link(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=100e3, nspan=2,
                  step_len=steps, edfa_gain=True)
    plan = D.dbp_step_plan(100e3, 2, steps)
    K = (n - 1) // 2
    m = np.fft.fftfreq(n) * n
    taps = []
    for d, _ in plan:
        Hinv = np.exp(-1j * BETA2 * (2 * np.pi * m * fs / n) ** 2 * d / 2)
        taps.append(np.array([np.sum(Hinv * np.exp(2j * np.pi * m * k / n)) / n for k in range(-K, K + 1)]))
    c = np.array([D.kerr_coef(d, z0, ALPHA, GAMMA) for d, z0 in plan])
    r = synth.complex_normal(1, n) * math.sqrt(0.03)
    np.testing.assert_allclose(L.ldbp_forward(r, taps, c), S.fft_dbp(r, link), atol=1e-12)


def test_ls_initialised_ldbp_approaches_dbp_with_many_taps():
    # More taps per step -> closer to FFT-DBP (truncation error shrinks); a sign error in xi would not converge.
    nsym = 256
    n = 2 * nsym
    fs = 21.4e9
    steps = D.log_steps(100e3, 2, ALPHA)
    link = S.Link(fs=fs, alpha=ALPHA, beta2=BETA2, gamma=GAMMA, span_len=100e3, nspan=2,
                  step_len=steps, edfa_gain=True)
    from oracle import txrx as X
    s = X.qam16(synth.qam16_indices(2, nsym))
    r = X.tx_shape(s, 2, 1e-3, 10.7e9)
    ref = S.fft_dbp(r, link)
    errs = []
    for T in (9, 41, 101):
        taps, c = D.init_asymmetric(100e3, 2, steps, T, fs, ALPHA, BETA2, GAMMA, method="truncate", N=n)
        errs.append(np.linalg.norm(L.ldbp_forward(r, taps, c) - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


@pytest.mark.parametrize("key", ["t_cd_10g7", "t_cd_32g"])
def test_t_cd_printed_values(key):
    g = GOLD[key]
    v = U.t_cd(U.beta2_from_ps2_per_km(g["beta2_ps2_per_km"]), g["delta_f"], g["length_m"], g["fs"])
    assert abs(v - g["value"]) <= g["tolerance"]


def test_total_taps_of_cascade():
    # Sec. V-A: the overall impulse response of 13 five-tap and 12 three-tap filters has 77 taps.
    g = GOLD["total_taps_77"]
    h = np.array([1.0])
    for T in [5] * g["n5"] + [3] * g["n3"]:
        h = np.convolve(h, np.ones(T))
    assert h.shape[0] == g["value"]


def test_rm_arithmetic():
    g = GOLD["rm_counts"]
    assert g["kerr_rm_per_step"] * g["steps"] == g["kerr_total"]
    n = 2048
    assert abs(n * (4 * math.log2(n) + 4) / (n - 69) - g["fd_eq_approx"]) < 1.0


def test_example2_pruning_event_count():
    g = GOLD["example2"]
    ev = TR.pruning_events(g["t_init"], g["t_final"])
    assert len(ev) == g["n_events"]
    assert TR.active_lengths(g["t_init"], ev, len(ev)) == g["t_final"]
    assert sorted(set(ev)) == list(range(5)) and all(ev.count(i) == 2 for i in range(5))


def test_pruning_schedule_front_loaded_and_masks():
    ev = TR.pruning_events([25] * 50, [3] * 50)
    assert len(ev) == 550
    its = TR.pruning_iterations(len(ev), 5000)             # events in the first 20% (reading R9)
    assert its == sorted(its) and its[-1] == 1000
    assert sum(1 for t in its if t < 500) > sum(1 for t in its if t >= 500)
    its = TR.pruning_iterations(len(ev), 5000, 0.6)
    assert its == sorted(its) and its[-1] == 3000
    assert sum(1 for t in its if t < 1500) > sum(1 for t in its if t >= 1500)
    h = [np.arange(1, 8, dtype=np.complex128)]
    np.testing.assert_allclose(TR.mask_taps(h, [3])[0], [0, 0, 3, 4, 5, 0, 0])


def test_adam_first_step_is_lr_times_sign():
    opt = TR.Adam(3, lr=1e-3)
    th = np.zeros(3)
    g = np.array([5.0, -0.01, 2.0])
    th1 = opt.step(th, g)
    np.testing.assert_allclose(th1, -1e-3 * np.sign(g), rtol=1e-5)


def test_adam_minimises_quadratic():
    opt = TR.Adam(2, lr=0.05)
    th = np.array([3.0, -2.0])
    for _ in range(2000):
        th = opt.step(th, 2 * (th - np.array([1.0, 0.5])))
    np.testing.assert_allclose(th, [1.0, 0.5], atol=1e-2)


def test_inband_fit_reduces_to_full_band_and_improves_band_error():
    xi, T = 0.497, 9
    np.testing.assert_allclose(D.ls_taps_inband(xi, T, 1.1 * np.pi / 2, mu=1.0), D.ls_taps(xi, T), atol=1e-12)
    w = 2 * np.pi * np.arange(-2048, 2049) / 4096
    band = np.abs(w) <= 1.1 * np.pi / 2
    k = np.arange(-(T // 2), T // 2 + 1)

    def band_err(h):
        return np.max(np.abs(np.exp(-1j * np.outer(w[band], k)) @ h - np.exp(1j * xi * w[band] ** 2)))

    hb = D.ls_taps_inband(xi, T, 1.1 * np.pi / 2)
    assert band_err(hb) < 0.2 * band_err(D.ls_taps(xi, T))
    # out-of-band gain stays bounded (no blow-up of the cascade)
    assert np.max(np.abs(np.exp(-1j * np.outer(w, k)) @ hb)) < 2.0


def _mo_case(M, T, fs=21.4e9, rho=2, rolloff=0.1):
    ds = [80e3 * (1.0 + 0.1 * (i % 3)) for i in range(M)]
    xis = [D.xi_of(d, BETA2, fs) for d in ds]
    edge = np.pi * (1.0 + rolloff) / rho
    return xis, edge


def test_multi_objective_single_filter_runs_give_individual_fits():
    """Runs of one filter only (max_window = 1): each filter's weighted LS problem is its own in-band fit
    (Sec. VI-B, first line of eq. objectives), whatever the starting values."""
    xis, edge = _mo_case(4, 7)
    start = [np.full(7, 0.1 + 0.2j) for _ in xis]
    out = D.multi_objective_ls(start, xis, edge, max_window=1, sweeps=1, N=1024)
    for h, xi in zip(out, xis):
        np.testing.assert_allclose(h, D.ls_taps_inband(xi, 7, edge, 1e-3, N=1024), rtol=1e-10, atol=1e-13)


def test_multi_objective_descends_and_ends_block_stationary():
    """Each update solves its weighted LS problem exactly, so the total objective (eq. objectives,
    all weights 1) never rises over the sweeps, and after the last update the last filter is a
    stationary point of the total objective: its central-difference derivative along random
    complex directions vanishes relative to the curvature."""
    M, T = 5, 5
    xis, edge = _mo_case(M, T)
    start = [D.ls_taps_inband(xi, T, edge, 1e-3, N=1024) for xi in xis]
    totals = [D.multi_objective_total(start, xis, edge)]
    hs = start
    for _ in range(3):
        hs = D.multi_objective_ls(hs, xis, edge, sweeps=1)
        totals.append(D.multi_objective_total(hs, xis, edge))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(totals, totals[1:]))
    assert totals[-1] < 0.7 * totals[0]
    g = np.random.Generator(np.random.PCG64(11))
    for _ in range(3):
        v = g.standard_normal(T) + 1j * g.standard_normal(T)
        eps = 1e-4

        def J(t):
            hh = list(hs)
            hh[-1] = hs[-1] + t * v
            return D.multi_objective_total(hh, xis, edge)
        j0, jp, jm = J(0.0), J(eps), J(-eps)
        slope = (jp - jm) / (2 * eps)
        curv = (jp - 2 * j0 + jm) / eps ** 2
        assert curv > 0
        assert abs(slope) <= 1e-6 * curv
