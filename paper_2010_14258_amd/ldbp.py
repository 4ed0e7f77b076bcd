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


def _plan(plan, guard: bool = False) -> Optional[N.LdbpPlan]:
    """None, an LdbpPlan, or a tuple (steps_per_pass, chunks[, outputs_per_thread[, symmetric[, one_stream]]]);
    guard adds LDBP_PLAN_GUARD (the forward's non-finite check)."""
    if plan is None:
        return N.LdbpPlan(0, 0, 0, N.LDBP_PLAN_GUARD) if guard else None
    if isinstance(plan, N.LdbpPlan):
        return N.LdbpPlan(plan.steps_per_pass, plan.chunks, plan.outputs_per_thread,
                          plan.flags | (N.LDBP_PLAN_GUARD if guard else 0))
    vals = list(plan) + [0] * (5 - len(plan))
    s, ch, rb, sym, one = vals[:5]
    flags = (N.LDBP_PLAN_SYMMETRIC if sym else 0) | (N.LDBP_PLAN_ONE_STREAM if one else 0) | \
        (N.LDBP_PLAN_GUARD if guard else 0)
    return N.LdbpPlan(int(s), int(ch), int(rb), flags)


def _shape(x: torch.Tensor, npol: int):
    if npol == 1:
        if x.dim() != 2:
            raise ValueError("x must be [nwave, n] for npol = 1")
        return x.shape[0], x.shape[1]
    if x.dim() != 3 or x.shape[2] != 2:
        raise ValueError("x must be [nwave, n, 2] for npol = 2")
    return x.shape[0], x.shape[1]


def ldbp_forward_workspace_size(x: torch.Tensor, ntap: Sequence[int], npol: int = 1, ckpt=None,
                                ckpt_every: int = 0, plan=None, guard: bool = False) -> int:
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    nt = N.i32_array(ntap)
    out = ctypes.c_size_t(0)
    pl = _plan(plan, guard)
    N.check(lib.ldbp_forward_workspace_size(code, npol, nwave, n, len(ntap), nt, _ptr(ckpt), int(ckpt_every),
                                            ctypes.byref(pl) if pl is not None else None, ctypes.byref(out)))
    return int(out.value)


def ldbp_forward_plan_query(dtype: int, npol: int, nwave: int, n: int, ntap: Sequence[int], ckpt_every: int = 0,
                            plan=None):
    """(passes, shortest tile length, most steps fused in a pass) of the forward's execution plan."""
    lib = N.load()
    a, b, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    pl = _plan(plan)
    N.check(lib.ldbp_forward_plan_query(dtype, npol, nwave, n, len(ntap), N.i32_array(ntap), int(ckpt_every),
                                        ctypes.byref(pl) if pl is not None else None, ctypes.byref(a),
                                        ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def ldbp_forward(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], npol: int = 1,
                 y: Optional[torch.Tensor] = None, ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                 plan=None, ws: Optional[torch.Tensor] = None, stream=None, guard: bool = False) -> torch.Tensor:
    """y = f_theta(x): l steps of circular FIR + Kerr phase (eq. model).  Returns y.

    guard: non-finite guard (LDBP_PLAN_GUARD): the call synchronises the stream and raises LdbpError
    with status LDBP_ENONFINITE when an output is a NaN or an infinity (y is written either way)."""
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
    pl = _plan(plan, guard)
    nt = N.i32_array(ntap)
    if ws is None:
        need = ldbp_forward_workspace_size(x, ntap, npol, ckpt, ckpt_every, plan, guard)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device) if need > 0 else None
    st = lib.ldbp_forward(code, npol, nwave, n, len(ntap), nt, _ptr(taps), _ptr(c), _ptr(x), _ptr(y),
                          _ptr(ckpt), int(ckpt_every), ctypes.byref(pl) if pl is not None else None,
                          _ptr(ws), ws.numel() if ws is not None else 0, stream_handle(stream, x.device))
    N.check(st)
    return y


def ldbp_forward_noalloc(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], y: torch.Tensor,
                         npol: int = 1, ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0, plan=None,
                         stream=None, guard: bool = False) -> torch.Tensor:
    """``ldbp_forward`` through the entry point that allocates nothing: the caller passes y (and ckpt), and
    the intermediate signal comes from the library's static device scratch (at most
    LDBP_NOALLOC_SCRATCH_BYTES; larger calls raise LdbpError with LDBP_EWORKSPACE).  Always one stream;
    calls that overlap on one device share the scratch and race."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    _check_dev("y", y, x.dtype)
    if taps.numel() != sum(int(t) for t in ntap) or c.numel() != len(ntap):
        raise ValueError("taps/c sizes do not match ntap")
    if ckpt is not None:
        _check_dev("ckpt", ckpt, x.dtype)
    pl = _plan(plan, guard)
    st = lib.ldbp_forward_noalloc(code, npol, nwave, n, len(ntap), N.i32_array(ntap), _ptr(taps), _ptr(c), _ptr(x),
                                  _ptr(y), _ptr(ckpt), int(ckpt_every), ctypes.byref(pl) if pl is not None else None,
                                  stream_handle(stream, x.device))
    N.check(st)
    return y


def ldbp_backward_workspace_size(x: torch.Tensor, ntap: Sequence[int], npol: int = 1, ckpt=None,
                                 ckpt_every: int = 0) -> int:
    lib = N.load()
    nwave, n = _shape(x, npol)
    out = ctypes.c_size_t(0)
    N.check(lib.ldbp_backward_workspace_size(_code(x), npol, nwave, n, len(ntap), N.i32_array(ntap), _ptr(ckpt),
                                             int(ckpt_every), ctypes.byref(out)))
    return int(out.value)


def ldbp_backward(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], gy: torch.Tensor,
                  npol: int = 1, ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0, need_gx: bool = True,
                  symmetric: bool = False, ws: Optional[torch.Tensor] = None, stream=None,
                  one_stream: bool = False):
    """Adjoint of ``ldbp_forward``: returns (gx or None, gtaps, gc) for dL/dy = gy (G = dL/dRe + j dL/dIm).

    symmetric: the taps satisfy h_{-k} = h_k; the FIR products are evaluated folded and gtaps is the
    gradient projected on symmetric filters ((dL/dh_k + dL/dh_{-k}) / 2 in both entries).
    one_stream: keep every launch on `stream` (by default the library may run half the batch on a
    second stream of its own, forked from and joined back into `stream`)."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    for name, t in (("x", x), ("gy", gy)):
        _check_dev(name, t, x.dtype)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    if ckpt is not None:
        _check_dev("ckpt", ckpt, x.dtype)
    gx = torch.empty_like(x) if need_gx else None
    gtaps = torch.empty_like(taps)
    gc = torch.empty_like(c)
    if ws is None:
        need = ldbp_backward_workspace_size(x, ntap, npol, ckpt, ckpt_every)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    pl = N.LdbpPlan(0, 0, 0, (N.LDBP_PLAN_SYMMETRIC if symmetric else 0) |
                    (N.LDBP_PLAN_ONE_STREAM if one_stream else 0))
    st = lib.ldbp_backward(code, npol, nwave, n, len(ntap), N.i32_array(ntap), _ptr(taps), _ptr(c), _ptr(x),
                           _ptr(ckpt), int(ckpt_every), _ptr(gy), _ptr(gx), _ptr(gtaps), _ptr(gc), ctypes.byref(pl),
                           _ptr(ws), ws.numel(), stream_handle(stream, x.device))
    N.check(st)
    return gx, gtaps, gc


def num_checkpoints(nstep: int, ckpt_every: int) -> int:
    """Checkpoint slots ldbp_forward writes for blocks of ``ckpt_every`` steps."""
    return 0 if ckpt_every <= 0 else max(0, -(-nstep // ckpt_every) - 1)


class LDBPFunction(torch.autograd.Function):
    """y = f_theta(x) with the hand-written adjoint; checkpoints every ``ckpt_every`` steps.

    apply(x, taps, c, ntap, npol, ckpt_every) -> y
    """

    @staticmethod
    def forward(ctx, x, taps, c, ntap, npol=1, ckpt_every=5):
        ntap = [int(t) for t in ntap]
        S = max(1, min(int(ckpt_every), len(ntap)))
        nslot = num_checkpoints(len(ntap), S)
        ckpt = torch.empty((max(nslot, 1),) + tuple(x.shape), dtype=x.dtype, device=x.device) if nslot else None
        # the backward reads the tensors the forward computed on: save the contiguous copies
        x, taps, c = x.contiguous(), taps.contiguous(), c.contiguous()
        y = ldbp_forward(x, taps, c, ntap, npol=npol, ckpt=ckpt, ckpt_every=S if ckpt is not None else 0,
                         plan=(S, 0) if ckpt is None else None)
        ctx.save_for_backward(x, taps, c, ckpt if ckpt is not None else torch.empty(0, device=x.device))
        ctx.ntap, ctx.npol, ctx.S, ctx.has_ckpt = ntap, npol, S, ckpt is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, taps, c, ckpt = ctx.saved_tensors
        gx, gt, gc = ldbp_backward(x, taps, c, ctx.ntap, gy.contiguous(), npol=ctx.npol,
                                   ckpt=ckpt if ctx.has_ckpt else None, ckpt_every=ctx.S,
                                   need_gx=ctx.needs_input_grad[0])
        return gx, gt, gc, None, None, None
