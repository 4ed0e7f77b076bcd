"""Python binding of the generalised ESSM entry points (argument marshalling only).

The generalised enhanced SSM is LDBP whose nonlinear steps filter the power before the phase
(Sec. III-D, eq. nl_filtered with a real filter per step): y_j = u_j exp(j c_i sum_k eta_k |u_{j-k}|^2).
Layouts as in ``ldbp``; ``eta`` is a real tensor (float32 for complex64, float64 for complex128)
holding the filters back to back, ``nl_ntap`` their odd lengths.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _native as N
from .ldbp import _check_dev, _code, _plan, _ptr, _real_dtype, _shape, stream_handle


def _check_model(ntap, nl_ntap, taps, c, eta):
    if len(nl_ntap) != len(ntap):
        raise ValueError("nl_ntap must have one entry per step")
    if (taps.numel() != sum(int(t) for t in ntap) or c.numel() != len(ntap)
            or eta.numel() != sum(int(t) for t in nl_ntap)):
        raise ValueError("taps/c/eta sizes do not match ntap/nl_ntap")


def essm_forward_workspace_size(x: torch.Tensor, ntap: Sequence[int], nl_ntap: Sequence[int], npol: int = 1,
                                ckpt=None, ckpt_every: int = 0, plan=None) -> int:
    lib = N.load()
    nwave, n = _shape(x, npol)
    out = ctypes.c_size_t(0)
    pl = _plan(plan)
    N.check(lib.essm_forward_workspace_size(_code(x), npol, nwave, n, len(ntap), N.i32_array(ntap),
                                            N.i32_array(nl_ntap), _ptr(ckpt), int(ckpt_every),
                                            ctypes.byref(pl) if pl is not None else None, ctypes.byref(out)))
    return int(out.value)


def essm_forward_plan_query(dtype: int, npol: int, nwave: int, n: int, ntap: Sequence[int], nl_ntap: Sequence[int],
                            ckpt_every: int = 0, plan=None):
    """(passes, shortest tile length, most steps fused in a pass) of the forward's execution plan."""
    lib = N.load()
    a, b, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    pl = _plan(plan)
    N.check(lib.essm_forward_plan_query(dtype, npol, nwave, n, len(ntap), N.i32_array(ntap), N.i32_array(nl_ntap),
                                        int(ckpt_every), ctypes.byref(pl) if pl is not None else None,
                                        ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def essm_forward(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, eta: torch.Tensor, ntap: Sequence[int],
                 nl_ntap: Sequence[int], npol: int = 1, y: Optional[torch.Tensor] = None,
                 ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0, plan=None,
                 ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = f_theta(x) with filtered nonlinear steps.  Returns y."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    _check_dev("eta", eta, _real_dtype(code))
    _check_model(ntap, nl_ntap, taps, c, eta)
    if y is None:
        y = torch.empty_like(x)
    _check_dev("y", y, x.dtype)
    if ckpt is not None:
        _check_dev("ckpt", ckpt, x.dtype)
    pl = _plan(plan)
    if ws is None:
        need = essm_forward_workspace_size(x, ntap, nl_ntap, npol, ckpt, ckpt_every, plan)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device) if need > 0 else None
    N.check(lib.essm_forward(code, npol, nwave, n, len(ntap), N.i32_array(ntap), N.i32_array(nl_ntap), _ptr(taps),
                             _ptr(c), _ptr(eta), _ptr(x), _ptr(y), _ptr(ckpt), int(ckpt_every),
                             ctypes.byref(pl) if pl is not None else None, _ptr(ws),
                             ws.numel() if ws is not None else 0, stream_handle(stream, x.device)))
    return y


def essm_backward_workspace_size(x: torch.Tensor, ntap: Sequence[int], nl_ntap: Sequence[int], npol: int = 1,
                                 ckpt=None, ckpt_every: int = 0) -> int:
    lib = N.load()
    nwave, n = _shape(x, npol)
    out = ctypes.c_size_t(0)
    N.check(lib.essm_backward_workspace_size(_code(x), npol, nwave, n, len(ntap), N.i32_array(ntap),
                                             N.i32_array(nl_ntap), _ptr(ckpt), int(ckpt_every), ctypes.byref(out)))
    return int(out.value)


def essm_backward(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, eta: torch.Tensor, ntap: Sequence[int],
                  nl_ntap: Sequence[int], gy: torch.Tensor, npol: int = 1, ckpt: Optional[torch.Tensor] = None,
                  ckpt_every: int = 0, need_gx: bool = True, symmetric: bool = False,
                  ws: Optional[torch.Tensor] = None, stream=None, one_stream: bool = False):
    """Adjoint of ``essm_forward``: returns (gx or None, gtaps, gc, geta) for dL/dy = gy.

    symmetric: the FIR taps satisfy h_{-k} = h_k (folded evaluation; gtaps projected on symmetric filters)."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    for name, t in (("x", x), ("gy", gy)):
        _check_dev(name, t, x.dtype)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    _check_dev("eta", eta, _real_dtype(code))
    _check_model(ntap, nl_ntap, taps, c, eta)
    if ckpt is not None:
        _check_dev("ckpt", ckpt, x.dtype)
    gx = torch.empty_like(x) if need_gx else None
    gtaps, gc, geta = torch.empty_like(taps), torch.empty_like(c), torch.empty_like(eta)
    if ws is None:
        ws = torch.empty(essm_backward_workspace_size(x, ntap, nl_ntap, npol, ckpt, ckpt_every), dtype=torch.uint8,
                         device=x.device)
    pl = N.LdbpPlan(0, 0, 0, (N.LDBP_PLAN_SYMMETRIC if symmetric else 0) |
                    (N.LDBP_PLAN_ONE_STREAM if one_stream else 0))
    N.check(lib.essm_backward(code, npol, nwave, n, len(ntap), N.i32_array(ntap), N.i32_array(nl_ntap), _ptr(taps),
                              _ptr(c), _ptr(eta), _ptr(x), _ptr(ckpt), int(ckpt_every), _ptr(gy), _ptr(gx),
                              _ptr(gtaps), _ptr(gc), _ptr(geta), ctypes.byref(pl), _ptr(ws), ws.numel(),
                              stream_handle(stream, x.device)))
    return gx, gtaps, gc, geta


class ESSMFunction(torch.autograd.Function):
    """y = f_theta(x) of the generalised ESSM with the hand-written adjoint; checkpoints every
    ``ckpt_every`` steps.  Gradients flow to x, taps, c and eta.

    apply(x, taps, c, eta, ntap, nl_ntap, npol, ckpt_every) -> y
    """

    @staticmethod
    def forward(ctx, x, taps, c, eta, ntap, nl_ntap, npol=1, ckpt_every=5):
        from .ldbp import num_checkpoints
        ntap = [int(t) for t in ntap]
        nl_ntap = [int(t) for t in nl_ntap]
        S = max(1, min(int(ckpt_every), len(ntap)))
        nslot = num_checkpoints(len(ntap), S)
        ckpt = torch.empty((nslot,) + tuple(x.shape), dtype=x.dtype, device=x.device) if nslot else None
        # the backward reads the tensors the forward computed on: save the contiguous copies
        x, taps, c, eta = x.contiguous(), taps.contiguous(), c.contiguous(), eta.contiguous()
        y = essm_forward(x, taps, c, eta, ntap, nl_ntap, npol=npol, ckpt=ckpt,
                         ckpt_every=S if ckpt is not None else 0, plan=(S, 0) if ckpt is None else None)
        ctx.save_for_backward(x, taps, c, eta, ckpt if ckpt is not None else torch.empty(0, device=x.device))
        ctx.ntap, ctx.nl_ntap, ctx.npol, ctx.S, ctx.has_ckpt = ntap, nl_ntap, npol, S, ckpt is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, taps, c, eta, ckpt = ctx.saved_tensors
        gx, gt, gc, ge = essm_backward(x, taps, c, eta, ctx.ntap, ctx.nl_ntap, gy.contiguous(), npol=ctx.npol,
                                       ckpt=ckpt if ctx.has_ckpt else None, ckpt_every=ctx.S,
                                       need_gx=ctx.needs_input_grad[0])
        return gx, gt, gc, ge, None, None, None, None
