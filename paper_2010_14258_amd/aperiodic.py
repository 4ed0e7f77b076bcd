"""Python binding of the aperiodic (streaming) forward (argument marshalling only) and a streaming
helper built on it.

The circular model of one block (Sec. III-B) becomes an equaliser for continuous data through
overlap-and-save (Sec. III-A): every FIR step is a full linear convolution, so an output depends only
on the inputs within P = sum_i (K_i + kappa_i) samples of it.

  edge "zero":  y [nwave, n(, 2)] = the model on x with zeros before and after it.
  edge "valid": y [nwave, n - 2P(, 2)] = the outputs at input positions P .. n - P - 1, the ones x
                determines whatever surrounds it.

``StreamEqualizer`` feeds a continuous stream chunk by chunk through the valid edge, keeping the last
2P input samples as context; the concatenated outputs equal the zero-edge forward of the whole
stream.  Buffer bookkeeping (the context copy) is device-memory plumbing; every step of the model
runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _native as N
from .ldbp import _check_dev, _code, _plan, _ptr, _real_dtype, _shape, stream_handle

EDGES = {"zero": N.LDBP_EDGE_ZERO, "valid": N.LDBP_EDGE_VALID}


def halo(ntap: Sequence[int], nl_ntap: Optional[Sequence[int]] = None) -> int:
    """P = sum_i (K_i + kappa_i): how far an output's dependence reaches."""
    P = sum((int(t) - 1) // 2 for t in ntap)
    if nl_ntap is not None:
        P += sum((int(t) - 1) // 2 for t in nl_ntap)
    return P


def _edge(edge) -> int:
    if edge not in EDGES:
        raise ValueError("edge must be 'zero' or 'valid'")
    return EDGES[edge]


def _nl(nl_ntap):
    return N.i32_array(nl_ntap) if nl_ntap is not None else None


def forward_aperiodic_workspace_size(x: torch.Tensor, ntap: Sequence[int], nl_ntap=None, npol: int = 1,
                                     edge: str = "zero", plan=None) -> int:
    lib = N.load()
    nwave, n = _shape(x, npol)
    out = ctypes.c_size_t(0)
    pl = _plan(plan)
    N.check(lib.ldbp_forward_aperiodic_workspace_size(_code(x), npol, nwave, n, len(ntap), N.i32_array(ntap),
                                                      _nl(nl_ntap), _edge(edge),
                                                      ctypes.byref(pl) if pl is not None else None,
                                                      ctypes.byref(out)))
    return int(out.value)


def forward_aperiodic(x: torch.Tensor, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], edge: str = "zero",
                      eta: Optional[torch.Tensor] = None, nl_ntap: Optional[Sequence[int]] = None, npol: int = 1,
                      y: Optional[torch.Tensor] = None, plan=None, ws: Optional[torch.Tensor] = None,
                      stream=None) -> torch.Tensor:
    """The aperiodic LDBP (eta None) or generalised ESSM forward.  Returns y."""
    lib = N.load()
    code = _code(x)
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    _check_dev("taps", taps, x.dtype)
    _check_dev("c", c, _real_dtype(code))
    if (eta is None) != (nl_ntap is None):
        raise ValueError("eta and nl_ntap go together")
    if eta is not None:
        _check_dev("eta", eta, _real_dtype(code))
        if len(nl_ntap) != len(ntap) or eta.numel() != sum(int(t) for t in nl_ntap):
            raise ValueError("eta size does not match nl_ntap")
    if taps.numel() != sum(int(t) for t in ntap) or c.numel() != len(ntap):
        raise ValueError("taps/c sizes do not match ntap")
    P = halo(ntap, nl_ntap)
    nout = n if edge == "zero" else n - 2 * P
    if nout < 1:
        raise ValueError(f"n = {n} leaves no valid output (2P = {2 * P})")
    shape = (nwave, nout) if npol == 1 else (nwave, nout, 2)
    if y is None:
        y = torch.empty(shape, dtype=x.dtype, device=x.device)
    _check_dev("y", y, x.dtype)
    if tuple(y.shape) != shape:
        raise ValueError(f"y must have shape {shape}")
    pl = _plan(plan)
    if ws is None:
        need = forward_aperiodic_workspace_size(x, ntap, nl_ntap, npol, edge, plan)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device) if need > 0 else None
    N.check(lib.ldbp_forward_aperiodic(code, npol, nwave, n, len(ntap), N.i32_array(ntap), _nl(nl_ntap), _ptr(taps),
                                       _ptr(c), _ptr(eta), _ptr(x), _ptr(y), _edge(edge),
                                       ctypes.byref(pl) if pl is not None else None, _ptr(ws),
                                       ws.numel() if ws is not None else 0, stream_handle(stream, x.device)))
    return y


class StreamEqualizer:
    """Overlap-save equaliser of continuous streams: push chunks of [nwave, m(, 2)] samples, get the
    outputs whose context is complete; ``flush`` ends the streams (zeros after their last sample).
    The outputs, concatenated, are the zero-edge forward of the whole streams."""

    def __init__(self, taps: torch.Tensor, c: torch.Tensor, ntap: Sequence[int], eta: Optional[torch.Tensor] = None,
                 nl_ntap: Optional[Sequence[int]] = None, npol: int = 1, plan=None, stream=None):
        self.taps, self.c, self.ntap = taps, c, list(ntap)
        self.eta, self.nl_ntap = eta, (list(nl_ntap) if nl_ntap is not None else None)
        self.npol, self.plan, self.stream = npol, plan, stream
        self.P = halo(self.ntap, self.nl_ntap)
        self.ctx = None   # input samples whose outputs are pending, plus P samples of history

    def _cat(self, chunk: torch.Tensor) -> torch.Tensor:
        if self.ctx is None:
            # P zeros before the first sample: the stream is zero before it starts
            shape = list(chunk.shape)
            shape[1] = self.P
            self.ctx = torch.zeros(shape, dtype=chunk.dtype, device=chunk.device)
        return torch.cat([self.ctx, chunk], dim=1)

    def push(self, chunk: torch.Tensor) -> torch.Tensor:
        buf = self._cat(chunk)
        m = buf.shape[1]
        if m <= 2 * self.P:
            self.ctx = buf
            return buf[:, :0]
        y = forward_aperiodic(buf, self.taps, self.c, self.ntap, "valid", self.eta, self.nl_ntap, self.npol,
                              plan=self.plan, stream=self.stream)
        self.ctx = buf[:, m - 2 * self.P:].clone()
        return y

    def flush(self) -> torch.Tensor:
        if self.ctx is None:
            raise RuntimeError("nothing was pushed")
        shape = list(self.ctx.shape)
        shape[1] = self.P
        out = self.push(torch.zeros(shape, dtype=self.ctx.dtype, device=self.ctx.device))
        self.ctx = None
        return out
