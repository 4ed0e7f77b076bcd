"""Generalised enhanced split-step model (ESSM): LDBP whose nonlinear steps filter the power first.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The enhanced (filtered) SSM modifies the nonlinear step so that the phase at time j is a weighted sum
of the squared modulus at neighbouring times (Sec. III-D, eq. nl_filtered); the generalisation gives
every step its own real filter eta^(i) = (eta_-kappa_i, ..., eta_kappa_i) and optimises all of them
together with the linear steps.  With the FIR linear steps of LDBP (Sec. III-B) step i is

    u   = h^(i) * x                                   (circular, centred, as in oracle.ldbp)
    F_j = sum_{k=-kappa_i}^{kappa_i} eta^(i)_k P_{(j-k) mod n},   P = |u|^2
    y_j = u_j exp(j c_i F_j)

where c_i is the per-step nonlinear coefficient of LDBP (gamma L_eff with its sign, Remark 1) and
P is summed over both polarisations for npol = 2 (Manakov phase, as in oracle.ldbp).  eta^(i) = (1)
(kappa_i = 0) is exactly the LDBP step.

Array layout as in oracle.ldbp: [..., n] or [..., n, 2].

Pins (tests/test_oracle_essm.py): eta = (1) reproduces ldbp_forward / ldbp_grad; brute-force dense
real circulant for the phase filter on tiny n; the closed form for a constant-envelope signal; c = 0
removes the filters; the (c s, eta / s) rescaling invariance and the orthogonality of the gradient
to it; central finite differences for every parameter group and the input (npol 1 and 2).
"""
from __future__ import annotations

import numpy as np

from .ldbp import _time_axis, fir_circular, power


def filter_power(P: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """F_j = sum_k eta_k P_{(j-k) mod n} along the last axis (real circular filter of odd length)."""
    eta = np.asarray(eta, dtype=np.float64)
    assert eta.shape[0] % 2 == 1, "filter length must be odd (2 kappa + 1)"
    kap = (eta.shape[0] - 1) // 2
    F = np.zeros(P.shape, dtype=np.float64)
    for k in range(-kap, kap + 1):
        F = F + eta[kap + k] * np.roll(P, k, axis=-1)   # np.roll(P, k)[j] = P[j - k]
    return F


def filtered_kerr(u: np.ndarray, c: float, eta: np.ndarray, npol: int = 1) -> np.ndarray:
    """y_j = u_j exp(j c sum_k eta_k |u_{j-k}|^2) (eq. nl_filtered with per-step filter)."""
    F = filter_power(power(u, npol), eta)
    rot = np.exp(1j * c * F)
    if npol == 2:
        rot = rot[..., None]
    return u * rot


def essm_forward(x: np.ndarray, taps, c, eta, npol: int = 1, return_all: bool = False):
    """l steps of circular FIR followed by the filtered nonlinear phase.

    taps: l odd-length complex vectors; c: l reals; eta: l odd-length real vectors.
    Returns y, or (y, ys, us) as oracle.ldbp.ldbp_forward.
    """
    x = np.asarray(x, dtype=np.complex128)
    c = np.asarray(c, dtype=np.float64)
    assert len(taps) == c.shape[0] == len(eta)
    ys, us = [x], []
    cur = x
    for i in range(len(taps)):
        u = fir_circular(cur, taps[i], npol)
        cur = filtered_kerr(u, c[i], eta[i], npol)
        us.append(u)
        ys.append(cur)
    if return_all:
        return cur, ys, us
    return cur


def phase_filter_matrix(eta: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n real matrix of the phase filter: row j holds eta_k in column (j-k) mod n (brute force)."""
    eta = np.asarray(eta, dtype=np.float64)
    kap = (eta.shape[0] - 1) // 2
    E = np.zeros((n, n), dtype=np.float64)
    for j in range(n):
        for k in range(-kap, kap + 1):
            E[j, (j - k) % n] += eta[kap + k]
    return E


def essm_grad(x: np.ndarray, taps, c, eta, gy: np.ndarray, npol: int = 1):
    """Adjoint of ``essm_forward`` for a real loss with dL/dy = gy (G = dL/dRe + j dL/dIm).

    The chain rule step by step in reverse (the paper gives none):
      filtered phase  y = u e^{j phi}, phi = c F, F = eta * P, P = |u|^2:
            q_j    = Im(G_y,j conj(y_j))              dL/dphi_j (summed over polarisations)
            dc     = sum_j q_j F_j
            deta_k = c sum_j q_j P_{j-k}
            r_m    = c sum_k eta_k q_{m+k}            dL/dP_m
            G_u    = G_y e^{-j phi} + 2 r u
      FIR  as oracle.ldbp.ldbp_grad.
    Returns (gx, gtaps (list), gc, geta (list)).
    """
    c = np.asarray(c, dtype=np.float64)
    y, ys, us = essm_forward(x, taps, c, eta, npol, return_all=True)
    G = np.asarray(gy, dtype=np.complex128)
    ax = _time_axis(npol)
    L = len(taps)
    gtaps, geta = [None] * L, [None] * L
    gc = np.zeros(L, dtype=np.float64)
    for i in range(L - 1, -1, -1):
        u, yi, xin = us[i], ys[i + 1], ys[i]
        e = np.asarray(eta[i], dtype=np.float64)
        kap = (e.shape[0] - 1) // 2
        P = power(u, npol)
        F = filter_power(P, e)
        q = (G * np.conj(yi)).imag
        if npol == 2:
            q = q.sum(axis=-1)
        gc[i] = float(np.sum(q * F))
        ge = np.zeros(e.shape[0], dtype=np.float64)
        r = np.zeros(q.shape, dtype=np.float64)
        for k in range(-kap, kap + 1):
            ge[kap + k] = c[i] * float(np.sum(q * np.roll(P, k, axis=-1)))   # P_{j-k}
            r = r + c[i] * e[kap + k] * np.roll(q, -k, axis=-1)               # q_{m+k}
        geta[i] = ge
        rot = np.exp(-1j * c[i] * F)
        r2 = 2.0 * r
        if npol == 2:
            rot = rot[..., None]
            r2 = r2[..., None]
        Gu = G * rot + r2 * u
        h = np.asarray(taps[i], dtype=np.complex128)
        K = (h.shape[0] - 1) // 2
        gh = np.zeros(h.shape[0], dtype=np.complex128)
        Gx = np.zeros(Gu.shape, dtype=np.complex128)
        for k in range(-K, K + 1):
            gh[K + k] = np.sum(Gu * np.conj(np.roll(xin, k, axis=ax)))
            Gx = Gx + np.conj(h[K + k]) * np.roll(Gu, -k, axis=ax)
        gtaps[i] = gh
        G = Gx
    return G, gtaps, gc, geta
