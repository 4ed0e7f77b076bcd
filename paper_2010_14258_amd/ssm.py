"""Python binding of the split-step channel simulator and FFT-DBP (argument marshalling only).

All units are SI.  ``Link`` mirrors the C ``ssm_link``; waveforms are complex
tensors [nwave, n] or [nwave, n, 2] (Manakov) on the GPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

from . import _native as N
from .ldbp import _check_dev, _code, _ptr, _shape, stream_handle


@dataclass
class Link:
    fs: float
    alpha: float
    beta2: float
    gamma: float
    span_len: float
    nspan: int
    nstep: int
    step_len: Optional[Sequence[float]] = None   # per-span step lengths, propagation order; None = uniform
    edfa_gain: bool = True
    ase_var: float = 0.0
    kerr_scale: float = 1.0

    def to_c(self):
        arr = None
        if self.step_len is not None:
            arr = (ctypes.c_double * len(self.step_len))(*[float(v) for v in self.step_len])
        st = N.SsmLink(self.fs, self.alpha, self.beta2, self.gamma, self.span_len, self.kerr_scale, self.ase_var,
                       int(self.nspan), int(self.nstep),
                       ctypes.cast(arr, N.P_f64) if arr is not None else None, int(bool(self.edfa_gain)), 0)
        return st, arr   # keep arr alive while st is used


def ssm_workspace_size(x: torch.Tensor, link: Link, npol: int = 1) -> int:
    lib = N.load()
    nwave, n = _shape(x, npol)
    st, keep = link.to_c()
    out = ctypes.c_size_t(0)
    N.check(lib.ssm_workspace_size(_code(x), npol, nwave, n, ctypes.byref(st), ctypes.byref(out)))
    return int(out.value)


def ssm_channel(x: torch.Tensor, link: Link, noise: Optional[torch.Tensor] = None, npol: int = 1,
                y: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Split-step channel: per span N(delta) then D(delta) per step, amplifier gain and sqrt(ase_var) * noise."""
    lib = N.load()
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    if noise is not None:
        _check_dev("noise", noise, x.dtype)
        if noise.numel() != link.nspan * x.numel():
            raise ValueError("noise must hold nspan x nwave x n (x npol) samples")
    y = torch.empty_like(x) if y is None else y
    _check_dev("y", y, x.dtype)
    if ws is None:
        ws = torch.empty(ssm_workspace_size(x, link, npol), dtype=torch.uint8, device=x.device)
    st, keep = link.to_c()
    N.check(lib.ssm_channel(_code(x), npol, nwave, n, ctypes.byref(st), _ptr(x), _ptr(y), _ptr(noise), _ptr(ws),
                            ws.numel(), stream_handle(stream, x.device)))
    return y


def fft_dbp(r: torch.Tensor, link: Link, npol: int = 1, y: Optional[torch.Tensor] = None,
            ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """FFT digital backpropagation over the link (the channel's exact reverse without noise)."""
    lib = N.load()
    nwave, n = _shape(r, npol)
    _check_dev("r", r)
    y = torch.empty_like(r) if y is None else y
    _check_dev("y", y, r.dtype)
    if ws is None:
        ws = torch.empty(ssm_workspace_size(r, link, npol), dtype=torch.uint8, device=r.device)
    st, keep = link.to_c()
    N.check(lib.fft_dbp(_code(r), npol, nwave, n, ctypes.byref(st), _ptr(r), _ptr(y), _ptr(ws), ws.numel(),
                        stream_handle(stream, r.device)))
    return y


class SsmBatchPlan:
    """Owns a C ``ssm_batch_plan``: the split-step channel (dbp=False) or FFT-DBP (dbp=True) over
    `link` for waveforms of lengths `wave_len` (2^a 3^b 5^c) with `wave_nspan` spans each, packed back
    to back as one complex tensor [sum wave_len] (npol = 1) or [sum wave_len, 2] (npol = 2)."""

    def __init__(self, wave_len: Sequence[int], wave_nspan: Sequence[int], link: Link, dbp: bool,
                 dtype=torch.complex64, npol: int = 1):
        lib = N.load()
        self.dtype, self.npol = dtype, npol
        self.wave_len = [int(v) for v in wave_len]
        self.wave_nspan = [int(v) for v in wave_nspan]
        lens = (ctypes.c_int64 * len(self.wave_len))(*self.wave_len)
        st, keep = link.to_c()
        h = ctypes.c_void_p(0)
        code = N.LDBP_C64 if dtype == torch.complex64 else N.LDBP_C128
        N.check(lib.ssm_batch_plan_create(code, npol, len(self.wave_len), lens, N.i32_array(self.wave_nspan),
                                          ctypes.byref(st), int(bool(dbp)), ctypes.byref(h)))
        self._h = h
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        c, d = ctypes.c_int32(0), ctypes.c_int32(0)
        N.check(lib.ssm_batch_plan_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        self.total_samples, self.total_sample_steps = a.value, b.value
        self.max_steps, self.noise_slots = c.value, d.value

    def close(self):
        if self._h is not None and self._h.value:
            N.load().ssm_batch_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, noise: Optional[torch.Tensor] = None,
            stream=None) -> torch.Tensor:
        lib = N.load()
        _check_dev("x", x, self.dtype)
        if x.numel() != self.total_samples * self.npol:
            raise ValueError("x does not hold the plan's samples")
        y = torch.empty_like(x) if y is None else y
        _check_dev("y", y, self.dtype)
        if noise is not None:
            _check_dev("noise", noise, self.dtype)
            if noise.numel() < self.noise_slots * x.numel():
                raise ValueError("noise must hold noise_slots x the plan's samples")
        N.check(lib.ssm_batch_run(self._h, _ptr(x), _ptr(y), _ptr(noise), stream_handle(stream, x.device)))
        return y
