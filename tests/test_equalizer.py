"""Host logic of the LDBP / FFT-DBP equaliser: the fallback policy and its force switch (no GPU needed)."""
import math

import pytest
import torch

from paper_2010_14258_amd import equalizer as EQ
from paper_2010_14258_amd import ssm as SS


def _eq(ntap=(15, 15, 3), taps_fill=0.1, c_fill=-1e-3):
    taps = torch.full((sum(ntap),), taps_fill, dtype=torch.complex64)
    c = torch.full((len(ntap),), c_fill, dtype=torch.float32)
    link = SS.Link(fs=21.4e9, alpha=4.6e-5, beta2=-2.17e-26, gamma=1.3e-3, span_len=1e5, nspan=1, nstep=1)
    return EQ.Equalizer(taps=taps, c=c, ntap=list(ntap), link=link)


def test_force_switch_reads_the_environment():
    assert EQ.forced_by_env({}) is False
    assert EQ.forced_by_env({"LDBP_FORCE_FFT_DBP": "0"}) is False
    assert EQ.forced_by_env({"LDBP_FORCE_FFT_DBP": ""}) is False
    assert EQ.forced_by_env({"LDBP_FORCE_FFT_DBP": "1"}) is True
    assert EQ.forced_by_env({"LDBP_FORCE_FFT_DBP": "yes"}) is True


def test_choose_policy_order():
    assert EQ.choose(True, True, True, 30.0, 20.0)[0] == "fft_dbp"
    assert EQ.choose(False, False, True, 30.0, 20.0) == ("fft_dbp", "no valid LDBP plan")
    assert EQ.choose(False, True, False, 30.0, 20.0) == ("fft_dbp", "non-finite LDBP parameters")
    assert EQ.choose(False, True, True, 19.9, 20.0) == ("fft_dbp", "LDBP below FFT-DBP on validation")
    assert EQ.choose(False, True, True, 20.0, 20.0)[0] == "ldbp"
    assert EQ.choose(False, True, True, None, 20.0)[0] == "ldbp"   # not validated yet
    assert EQ.choose(False, True, True, -math.inf, 20.0)[0] == "fft_dbp"


def test_equalizer_decisions_on_host_tensors(monkeypatch):
    """decide() uses only the library's host-side plan query and the parameter values."""
    monkeypatch.delenv("LDBP_FORCE_FFT_DBP", raising=False)
    r = torch.zeros((2, 4096), dtype=torch.complex64)
    eq = _eq()
    assert eq.decide(r)[0] == "ldbp"
    monkeypatch.setenv("LDBP_FORCE_FFT_DBP", "1")
    assert eq.decide(r) == ("fft_dbp", "forced")
    monkeypatch.delenv("LDBP_FORCE_FFT_DBP")
    bad = _eq(ntap=(15, 4, 3))            # an even filter length has no plan
    assert bad.decide(r) == ("fft_dbp", "no valid LDBP plan")
    nan = _eq(c_fill=float("nan"))
    assert nan.decide(r) == ("fft_dbp", "non-finite LDBP parameters")
    eq.ldbp_snr_db, eq.fft_dbp_snr_db = 25.0, 26.0
    assert eq.decide(r)[0] == "fft_dbp"
    eq.ldbp_snr_db = 27.0
    assert eq.decide(r)[0] == "ldbp"
