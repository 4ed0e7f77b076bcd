"""Aperiodic (streaming) LDBP and ESSM: the model without the circular boundary.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The circulant matrices of Sec. III-B describe one periodic block of n samples; continuous data is
processed in blocks with overlap-and-save, the block length n being chosen to keep that overhead
small (Sec. III-A).  The aperiodic model is the same stack with every FIR step a full linear
convolution of a signal that is zero outside its support:

    u_m = sum_{k=-K}^{K} h_k x_{m-k},      x_t = 0 outside the support of x,

so the support grows by K on each side per step; the (filtered) Kerr phase acts pointwise on u
(F_j = sum_k eta_k P_{j-k} with P = |u|^2 zero outside u's support, Sec. III-D) and leaves the
support unchanged.  With P_tot = sum_i (K_i + kappa_i), an output at time t depends only on inputs
at times t - P_tot .. t + P_tot.

  edge "zero":  the outputs at the n input times 0 .. n-1.
  edge "valid": the outputs at times P_tot .. n - P_tot - 1, which x determines whatever lies
                outside it (overlap-save: chunks of a stream passed with P_tot samples of context
                on each side give the stream's outputs exactly).

Array layout as in oracle.ldbp: [..., n] or [..., n, 2] (npol = 2, Manakov phase).

Pins (tests/test_oracle_aperiodic.py): brute-force rectangular Toeplitz matrices on tiny inputs;
the circular oracle on a zero-padded input (zero) and on the input itself (valid), both with LDBP
and filtered steps; the c = 0 cascade equals one linear convolution with the convolution of the
filters; shift equivariance; chunked valid outputs reproduce the whole stream.
"""
from __future__ import annotations

import numpy as np

from .ldbp import _time_axis, power


def _tslice(a: np.ndarray, lo: int, hi: int, npol: int) -> np.ndarray:
    """a[..., lo:hi] along the time axis."""
    if npol == 1:
        return a[..., lo:hi]
    return a[..., lo:hi, :]


def _zpad(a: np.ndarray, left: int, right: int, npol: int) -> np.ndarray:
    ax = _time_axis(npol) % a.ndim
    width = [(0, 0)] * a.ndim
    width[ax] = (left, right)
    return np.pad(a, width)


def fir_full(x: np.ndarray, h: np.ndarray, npol: int = 1) -> np.ndarray:
    """Full linear convolution along time: input support [0, n), output support [-K, n + K)."""
    h = np.asarray(h, dtype=np.complex128)
    K = (h.shape[0] - 1) // 2
    n = x.shape[_time_axis(npol)]
    X = _zpad(np.asarray(x, dtype=np.complex128), 2 * K, 2 * K, npol)  # X[t + 2K] = x_t
    u = 0
    for k in range(-K, K + 1):
        # u_m (array index a = m + K) = sum_k h_k x_{m-k} = sum_k h_k X[a + K - k]
        u = u + h[K + k] * _tslice(X, K - k, K - k + n + 2 * K, npol)
    return u


def filtered_phase_full(u: np.ndarray, c: float, eta, npol: int = 1) -> np.ndarray:
    """u_j exp(j c sum_k eta_k P_{j-k}) with P = |u|^2 zero outside u's support (eta = None: Kerr)."""
    P = power(u, npol)
    if eta is None:
        F = P
    else:
        eta = np.asarray(eta, dtype=np.float64)
        kap = (eta.shape[0] - 1) // 2
        m = P.shape[-1]
        Pp = np.pad(P, [(0, 0)] * (P.ndim - 1) + [(kap, kap)])  # Pp[j + kap] = P_j
        F = 0
        for k in range(-kap, kap + 1):
            F = F + eta[kap + k] * Pp[..., kap - k:kap - k + m]
    rot = np.exp(1j * c * F)
    if npol == 2:
        rot = rot[..., None]
    return u * rot


def halo(taps, eta=None) -> int:
    """P_tot = sum_i (K_i + kappa_i): how far an output's dependence reaches."""
    P = sum((len(h) - 1) // 2 for h in taps)
    if eta is not None:
        P += sum((len(e) - 1) // 2 for e in eta)
    return P


def forward_aperiodic(x: np.ndarray, taps, c, eta=None, edge: str = "zero", npol: int = 1) -> np.ndarray:
    """The aperiodic stack: l steps of full convolution followed by the (filtered) Kerr phase."""
    c = np.asarray(c, dtype=np.float64)
    cur = np.asarray(x, dtype=np.complex128)
    n = cur.shape[_time_axis(npol)]
    grown = 0
    for i in range(len(taps)):
        u = fir_full(cur, taps[i], npol)
        grown += (len(taps[i]) - 1) // 2
        cur = filtered_phase_full(u, c[i], None if eta is None else eta[i], npol)
    if edge == "zero":
        return _tslice(cur, grown, grown + n, npol)
    P = halo(taps, eta)
    assert n > 2 * P, "valid edge needs n > 2 P"
    return _tslice(cur, grown + P, grown + n - P, npol)


def toeplitz_full(h: np.ndarray, n: int) -> np.ndarray:
    """Dense (n + 2K) x n matrix of the full convolution: row a (time a - K), column t: h_{a - K - t}."""
    h = np.asarray(h, dtype=np.complex128)
    K = (h.shape[0] - 1) // 2
    M = np.zeros((n + 2 * K, n), dtype=np.complex128)
    for a in range(n + 2 * K):
        for t in range(n):
            k = a - K - t
            if -K <= k <= K:
                M[a, t] = h[K + k]
    return M
