"""Python binding of batched uneven LDBP inference (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _native as N
from .ldbp import _check_dev, _plan, _ptr, stream_handle


class BatchPlan:
    """Owns a C ``ldbp_batch_plan``: per-waveform lengths, step counts and tap counts."""

    def __init__(self, wave_len: Sequence[int], wave_nstep: Sequence[int], step_ntap: Sequence[int],
                 dtype=torch.complex64, npol: int = 1, plan=None):
        lib = N.load()
        self.dtype = dtype
        self.npol = npol
        code = N.LDBP_C64 if dtype == torch.complex64 else N.LDBP_C128
        self.wave_len = [int(v) for v in wave_len]
        self.wave_nstep = [int(v) for v in wave_nstep]
        self.step_ntap = [int(v) for v in step_ntap]
        lens = (ctypes.c_int64 * len(self.wave_len))(*self.wave_len)
        ns = N.i32_array(self.wave_nstep)
        nt = N.i32_array(self.step_ntap)
        pl = _plan(plan)
        h = ctypes.c_void_p(0)
        N.check(lib.ldbp_batch_plan_create(code, npol, len(self.wave_len), lens, ns, nt,
                                           ctypes.byref(pl) if pl is not None else None, ctypes.byref(h)))
        self._h = h
        a, b, c, d = (ctypes.c_int64(0) for _ in range(4))
        e, f = ctypes.c_int32(0), ctypes.c_int32(0)
        N.check(lib.ldbp_batch_plan_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                         ctypes.byref(e), ctypes.byref(f)))
        self.total_samples, self.total_sample_steps, self.total_taps, self.total_steps = a.value, b.value, c.value, d.value
        self.nitems, self.work = e.value, f.value

    def close(self):
        if self._h is not None and self._h.value:
            N.load().ldbp_batch_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, taps, c, x, y):
        rd = torch.float32 if self.dtype == torch.complex64 else torch.float64
        _check_dev("x", x, self.dtype)
        _check_dev("y", y, self.dtype)
        _check_dev("taps", taps, self.dtype)
        _check_dev("c", c, rd)
        if x.numel() != self.total_samples * self.npol or taps.numel() != self.total_taps or \
                c.numel() != self.total_steps:
            raise ValueError("packed array sizes do not match the plan")

    def forward(self, taps: torch.Tensor, c: torch.Tensor, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                graph: bool = False, stream=None) -> torch.Tensor:
        y = torch.empty_like(x) if y is None else y
        self._check(taps, c, x, y)
        lib = N.load()
        fn = lib.ldbp_batch_forward_graph if graph else lib.ldbp_batch_forward
        N.check(fn(self._h, _ptr(taps), _ptr(c), _ptr(x), _ptr(y), stream_handle(stream, x.device)))
        return y
