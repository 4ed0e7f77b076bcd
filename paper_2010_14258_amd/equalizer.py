"""Receiver-side equaliser: learned DBP with plain FFT-based DBP as the fallback.

LDBP (Sec. III-B) replaces the frequency-domain linear steps of digital backpropagation by short
learned FIR filters; FFT-DBP (Sec. III-A, the split-step method run backwards with the link's
parameters) needs no training and is the conventional method the learned one is judged against.
This module picks between the two per call:

  * ``LDBP_FORCE_FFT_DBP`` set to a non-empty value other than ``0`` routes every call to FFT-DBP;
  * a model with no valid execution plan (the library's plan query fails) or non-finite parameters
    routes to FFT-DBP;
  * after ``validate`` has measured both methods' effective SNR on labelled data, a learned model
    whose SNR is below FFT-DBP's routes to FFT-DBP;
  * otherwise LDBP runs with the library's non-finite guard; when its output holds a NaN or an
    infinity (status LDBP_ENONFINITE) the same input goes through FFT-DBP instead.

The decision itself (``choose``) is host logic; every computation runs in the library's kernels.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _native as N
from . import ldbp as L
from . import ssm as SS
from . import txrx as TX

FORCE_ENV = "LDBP_FORCE_FFT_DBP"


def forced_by_env(environ=None) -> bool:
    v = (os.environ if environ is None else environ).get(FORCE_ENV, "")
    return v.strip() not in ("", "0")


def choose(forced: bool, plan_ok: bool, params_finite: bool, ldbp_snr_db: Optional[float],
           fft_dbp_snr_db: Optional[float]):
    """('ldbp' | 'fft_dbp', reason) for one call; SNRs are None until validated."""
    if forced:
        return "fft_dbp", "forced"
    if not plan_ok:
        return "fft_dbp", "no valid LDBP plan"
    if not params_finite:
        return "fft_dbp", "non-finite LDBP parameters"
    if ldbp_snr_db is not None and fft_dbp_snr_db is not None and ldbp_snr_db < fft_dbp_snr_db:
        return "fft_dbp", "LDBP below FFT-DBP on validation"
    return "ldbp", "ldbp"


@dataclass
class Equalizer:
    """LDBP model (taps [sum ntap] complex, c [l] real, on the GPU) with its FFT-DBP fallback link."""
    taps: torch.Tensor
    c: torch.Tensor
    ntap: Sequence[int]
    link: SS.Link
    npol: int = 1
    symmetric: bool = False
    ldbp_snr_db: Optional[float] = None
    fft_dbp_snr_db: Optional[float] = None
    events: List[tuple] = field(default_factory=list)

    def plan_ok(self, r: torch.Tensor) -> bool:
        nwave, n = r.shape[0], r.shape[1]
        code = N.LDBP_C64 if r.dtype == torch.complex64 else N.LDBP_C128
        try:
            L.ldbp_forward_plan_query(code, self.npol, nwave, n, list(self.ntap),
                                      plan=(0, 0, 0, 1 if self.symmetric else 0))
        except N.LdbpError:
            return False
        return True

    def params_finite(self) -> bool:
        return bool(torch.isfinite(torch.view_as_real(self.taps)).all().item()) and \
            bool(torch.isfinite(self.c).all().item())

    def decide(self, r: torch.Tensor):
        return choose(forced_by_env(), self.plan_ok(r), self.params_finite(), self.ldbp_snr_db, self.fft_dbp_snr_db)

    def fft_dbp(self, r: torch.Tensor) -> torch.Tensor:
        return SS.fft_dbp(r, self.link, npol=self.npol)

    def ldbp(self, r: torch.Tensor, guard: bool = True) -> torch.Tensor:
        return L.ldbp_forward(r, self.taps, self.c, list(self.ntap), npol=self.npol,
                              plan=(0, 0, 0, 1 if self.symmetric else 0), guard=guard)

    def __call__(self, r: torch.Tensor):
        """Equalised waveforms and the path taken ('ldbp' or 'fft_dbp')."""
        path, why = self.decide(r)
        if path == "ldbp":
            try:
                return self.ldbp(r), "ldbp"
            except N.LdbpError as e:
                if e.status != N.LDBP_ENONFINITE:
                    raise
                why = "non-finite LDBP output"
        self.events.append(("fft_dbp", why))
        return self.fft_dbp(r), "fft_dbp"

    def validate(self, r: torch.Tensor, s: torch.Tensor, p_watt: torch.Tensor, rho: int, rs: float,
                 rolloff: float = 0.1):
        """Effective SNR [dB] of both methods on received waveforms r with transmitted symbols s (receiver
        DSP of Sec. IV-A/B: matched filter, genie phase, SNR = 1 / MSE)."""
        def snr(z):
            mse, _, _ = TX.rx_mse(z, s, p_watt, rho, rs, rolloff, npol=self.npol)
            m = float(mse.mean().item())
            return 10.0 * math.log10(1.0 / m) if m > 0 and math.isfinite(m) else -math.inf
        try:
            self.ldbp_snr_db = snr(self.ldbp(r, guard=False))
        except N.LdbpError:
            self.ldbp_snr_db = -math.inf
        self.fft_dbp_snr_db = snr(self.fft_dbp(r))
        return self.ldbp_snr_db, self.fft_dbp_snr_db
