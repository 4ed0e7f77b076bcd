"""Python binding of the LDBP C ABI (argument marshalling only).

Tensors are PyTorch CUDA (HIP) tensors used as device memory; every step of
the computation runs in the HIP kernels of ``libldbp.so``.  Waveform batches
are complex tensors of shape [nwave, n] (single polarisation) or
[nwave, n, 2] (dual polarisation, Manakov).  Filter taps are packed into one
complex vector, filter i holding ``ntap[i]`` centred taps (index K_i + k holds
h_k).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _native as N


def _code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return N.LDBP_C64
    if t.dtype == torch.complex128:
        return N.LDBP_C128
    raise TypeError(f"complex64 or complex128 expected, got {t.dtype}")


def _real_dtype(code: int):
    return torch.float32 if code == N.LDBP_C64 else torch.float64


def stream_handle(stream: Optional[torch.cuda.Stream] = None, device=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_dev(name: str, t: torch.Tensor, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _plan(plan) -> Optional[N.LdbpPlan]:
    if plan is None:
        return None
    if isinstance(plan, N.LdbpPlan):
        return plan
    s, ch = plan
    return N.LdbpPlan(int(s), int(ch), 0, 0)


def _shape(x: torch.Tensor, npol: int):
    if npol == 1:
        if x.dim() != 2:
            raise ValueError("x must be [nwave, n] for npol = 1")
        return x.shape[0], x.shape[1]
    if x.dim() != 3 or x.shape[2] != 2:
        raise ValueError("x must be [nwave, n, 2] for npol = 2")
    return x.shape[0], x.shape[1]


def ldbp_forward_workspace_size(x: torch.Tensor, ntap: Sequence[int], npol: int = 1, ckpt=None,
                                ckpt_every: int = 0, plan=None) -> int:
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    nt = N.i32_array(ntap)
    out = ctypes.c_size_t(0)
    pl = _plan(plan)
    N.check(lib.ldbp_forward_workspace_size(code, npol, nwave, n, len(ntap), nt, _ptr(ckpt), int(ckpt_every),
                                            ctypes.byref(pl) if pl is not None else None, ctypes.byref(out)))
    return int(out.value)


def ldbp_forward(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], npol: int = 1,
                 y: Optional[torch.Tensor] = None, ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                 plan=None, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = f_theta(x): l steps of circular FIR + Kerr phase (eq. model).  Returns y."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    if taps.numel() != sum(int(t) for t in ntap) or c.numel() != len(ntap):
        raise ValueError("taps/c sizes do not match ntap")
    if y is None:
        y = torch.empty_like(x)
    _check_dev("y", y, x.dtype)
    if ckpt is not None:
        _check_dev("ckpt", ckpt, x.dtype)
    pl = _plan(plan)
    nt = N.i32_array(ntap)
    if ws is None:
        need = ldbp_forward_workspace_size(x, ntap, npol, ckpt, ckpt_every, plan)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device) if need > 0 else None
    st = lib.ldbp_forward(code, npol, nwave, n, len(ntap), nt, _ptr(taps), _ptr(c), _ptr(x), _ptr(y),
                          _ptr(ckpt), int(ckpt_every), ctypes.byref(pl) if pl is not None else None,
                          _ptr(ws), ws.numel() if ws is not None else 0, stream_handle(stream, x.device))
    N.check(st)
    return y
