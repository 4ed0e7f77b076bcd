"""Python binding of the batched FFT, TX/RX DSP, random numbers and Adam (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _native as N
from .ldbp import _check_dev, _code, _ptr, _shape, stream_handle


def _ws(fn, *args) -> int:
    out = ctypes.c_size_t(0)
    N.check(fn(*args, ctypes.byref(out)))
    return int(out.value)


def _alloc(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def fft(x: torch.Tensor, inverse: bool = False, npol: int = 1, y: Optional[torch.Tensor] = None, stream=None):
    """Unnormalised DFT along the sample axis (natural order)."""
    lib = N.load()
    nwave, n = _shape(x, npol)
    _check_dev("x", x)
    y = torch.empty_like(x) if y is None else y
    ws = _alloc(_ws(lib.ldbp_fft_workspace_size, _code(x), npol, nwave, n), x.device)
    N.check(lib.ldbp_fft(_code(x), npol, nwave, n, _ptr(x), _ptr(y), int(inverse), _ptr(ws), ws.numel(),
                         stream_handle(stream, x.device)))
    return y


def tx_shape(sym_idx: torch.Tensor, p_watt: torch.Tensor, rho: int, rs: float, rolloff: float = 0.1,
             npol: int = 1, dtype=torch.complex64, stream=None) -> torch.Tensor:
    """16-QAM, RRC-shaped periodic waveform [nwave, rho*nsym(, 2)] from indices [nwave, nsym(, 2)]."""
    lib = N.load()
    code = N.LDBP_C64 if dtype == torch.complex64 else N.LDBP_C128
    _check_dev("sym_idx", sym_idx, torch.int32)
    _check_dev("p_watt", p_watt, torch.float64)
    nwave, nsym = sym_idx.shape[0], sym_idx.shape[1]
    shape = (nwave, rho * nsym) if npol == 1 else (nwave, rho * nsym, 2)
    x = torch.empty(shape, dtype=dtype, device=sym_idx.device)
    ws = _alloc(_ws(lib.tx_shape_workspace_size, code, npol, nwave, nsym, rho), x.device)
    N.check(lib.tx_shape(code, npol, nwave, nsym, rho, rs, rolloff, _ptr(sym_idx), _ptr(p_watt), _ptr(x), _ptr(ws),
                         ws.numel(), stream_handle(stream, x.device)))
    return x


def rx_lpf_decimate(y: torch.Tensor, n_out: int, npol: int = 1, stream=None) -> torch.Tensor:
    lib = N.load()
    nwave, n_in = _shape(y, npol)
    _check_dev("y", y)
    shape = (nwave, n_out) if npol == 1 else (nwave, n_out, 2)
    r = torch.empty(shape, dtype=y.dtype, device=y.device)
    ws = _alloc(_ws(lib.rx_lpf_decimate_workspace_size, _code(y), npol, nwave, n_in, n_out), y.device)
    N.check(lib.rx_lpf_decimate(_code(y), npol, nwave, n_in, n_out, _ptr(y), _ptr(r), _ptr(ws), ws.numel(),
                                stream_handle(stream, y.device)))
    return r


def tx_shape_symbols(sym: torch.Tensor, p_watt: torch.Tensor, rho: int, rs: float, rolloff: float = 0.1,
                     npol: int = 1, stream=None) -> torch.Tensor:
    """RRC-shaped periodic waveform [nwave, rho*nsym(, 2)] from complex symbols [nwave, nsym(, 2)]."""
    lib = N.load()
    _check_dev("sym", sym)
    _check_dev("p_watt", p_watt, torch.float64)
    code = _code(sym)
    nwave, nsym = sym.shape[0], sym.shape[1]
    shape = (nwave, rho * nsym) if npol == 1 else (nwave, rho * nsym, 2)
    x = torch.empty(shape, dtype=sym.dtype, device=sym.device)
    ws = _alloc(_ws(lib.tx_shape_workspace_size, code, npol, nwave, nsym, rho), x.device)
    N.check(lib.tx_shape_symbols(code, npol, nwave, nsym, rho, rs, rolloff, _ptr(sym), _ptr(p_watt), _ptr(x),
                                 _ptr(ws), ws.numel(), stream_handle(stream, x.device)))
    return x


def qam16_symbols(sym_idx: torch.Tensor, dtype=torch.complex64, stream=None) -> torch.Tensor:
    lib = N.load()
    _check_dev("sym_idx", sym_idx, torch.int32)
    s = torch.empty(sym_idx.shape, dtype=dtype, device=sym_idx.device)
    code = N.LDBP_C64 if dtype == torch.complex64 else N.LDBP_C128
    N.check(lib.qam16_symbols(code, sym_idx.numel(), _ptr(sym_idx), _ptr(s), stream_handle(stream, s.device)))
    return s


def rx_mse(z: torch.Tensor, sym: torch.Tensor, p_watt: torch.Tensor, rho: int, rs: float, rolloff: float = 0.1,
           npol: int = 1, want_grad: bool = False, want_shat: bool = False, stream=None):
    """Matched filter + downsampling + genie phase: returns (mse [nwave*npol] float64, s_hat or None, gz or None)."""
    lib = N.load()
    nwave, n = _shape(z, npol)
    nsym = sym.shape[1]
    _check_dev("z", z)
    _check_dev("sym", sym, z.dtype)
    _check_dev("p_watt", p_watt, torch.float64)
    mse = torch.empty(nwave * npol, dtype=torch.float64, device=z.device)
    shat = torch.empty_like(sym) if want_shat else None
    gz = torch.empty_like(z) if want_grad else None
    ws = _alloc(_ws(lib.rx_mse_workspace_size, _code(z), npol, nwave, nsym, rho), z.device)
    N.check(lib.rx_mse(_code(z), npol, nwave, nsym, rho, rs, rolloff, _ptr(z), _ptr(sym), _ptr(p_watt), _ptr(shat),
                       _ptr(mse), _ptr(gz), _ptr(ws), ws.numel(), stream_handle(stream, z.device)))
    return mse, shat, gz


def randbits(nwords: int, seed: int, stream_id: int, device="cuda", stream=None) -> torch.Tensor:
    lib = N.load()
    out = torch.empty(nwords, dtype=torch.int32, device=device)
    N.check(lib.ldbp_randbits(_ptr(out), nwords, int(seed), int(stream_id), stream_handle(stream, out.device)))
    return out


def randn(shape, seed: int, stream_id: int, dtype=torch.complex64, device="cuda", stream=None) -> torch.Tensor:
    lib = N.load()
    out = torch.empty(shape, dtype=dtype, device=device)
    code = N.LDBP_C64 if dtype == torch.complex64 else N.LDBP_C128
    N.check(lib.ldbp_randn(code, _ptr(out), out.numel(), int(seed), int(stream_id), stream_handle(stream, out.device)))
    return out


def sum_rows(x: torch.Tensor, rows: int, stream=None) -> torch.Tensor:
    """Sum over `rows` equal consecutive blocks of x (real or complex, contiguous), in the library's
    fixed order: returns x.view(rows, -1) summed over the first axis."""
    lib = N.load()
    rx = torch.view_as_real(x) if x.is_complex() else x
    _check_dev("x", rx)
    if rx.numel() % rows:
        raise ValueError("x does not split into rows")
    cols = rx.numel() // rows
    out = torch.empty(x.numel() // rows, dtype=x.dtype, device=x.device)
    ro = torch.view_as_real(out) if out.is_complex() else out
    code = N.LDBP_C64 if rx.dtype == torch.float32 else N.LDBP_C128
    N.check(lib.ldbp_sum_rows(code, _ptr(rx), _ptr(ro), rows, cols, stream_handle(stream, x.device)))
    return out


def adam_(theta: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int, lr: float = 1e-3,
          b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, mask: Optional[torch.Tensor] = None,
          mirror: Optional[torch.Tensor] = None, stream=None):
    """In-place Adam step on a real (float32/float64) or complex parameter tensor."""
    lib = N.load()
    comps = 2 if theta.is_complex() else 1
    rt = torch.view_as_real(theta) if comps == 2 else theta
    rg = torch.view_as_real(grad) if comps == 2 else grad
    for name, tt in (("theta", rt), ("grad", rg), ("m", m), ("v", v)):
        _check_dev(name, tt, rt.dtype)
    if mask is not None:
        _check_dev("mask", mask, rt.dtype)
    if mirror is not None:
        _check_dev("mirror", mirror, torch.int32)
    code = N.LDBP_C64 if rt.dtype == torch.float32 else N.LDBP_C128
    N.check(lib.ldbp_adam(code, _ptr(rt), _ptr(rg), _ptr(m), _ptr(v), _ptr(mask), _ptr(mirror), rt.numel(), comps,
                          lr, b1, b2, eps, int(t), stream_handle(stream, rt.device)))
