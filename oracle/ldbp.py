"""LDBP model: the parameterised split-step method of eq. (model), Sec. III-B, and its adjoint.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Model (eq. model with the FIR constraint of Sec. III-B and the per-step
nonlinear scaling of Remark 1):

    f_theta(x) = sigma_l(A^(l) ... sigma_1(A^(1) x))

  * A^(i) is circular convolution with a centred FIR filter of odd length
    T_i = 2 K_i + 1:  u_m = sum_{k=-K_i}^{K_i} h^(i)_k x_{(m-k) mod n}.
    (Reading of the circulant rows in Sec. III-B: h_0 sits on the diagonal, i.e.
    zero delay, consistent with the centred DTFT used for the filter design in
    Sec. IV-C.)  Taps are stored in full, index K_i + k holds h_k; symmetry, when
    wanted, is a property of the values, not of the storage.
  * sigma_i(u) = u exp(j c_i |u|^2), one real coefficient c_i per step; c_i is
    gamma * L_eff(delta_i) * eta^(i) with its sign (Remark 1, Sec. III-A).  A
    symmetric-SSM based model sets c_l = 0 (Sec. III-C).
  * Dual polarisation (Manakov, Sec. III-D names the coupled equations):
    arrays carry a trailing axis of length 2; both polarisations share the taps
    and the phase c_i (|u_x|^2 + |u_y|^2) rotates both.

Array layout: x has shape [..., n] (single polarisation) or [..., n, 2]
(``npol=2``); any leading axes are independent waveforms that share theta.

Pins (tests/test_oracle_ldbp.py): FFT circular convolution with asymmetric taps;
T = n inverse-DFT taps reproduce frequency-domain filtering (LDBP contains DBP);
c = 0 collapses to one filter equal to the convolution of all filters
(Sec. VI-C); |sigma(u)| = |u|; Remark 4 rescaling invariance; brute-force dense
circulant products for tiny n; central finite differences and a dot-product test
for the adjoint.
"""
from __future__ import annotations

import numpy as np


def _time_axis(npol: int) -> int:
    return -1 if npol == 1 else -2


def fir_circular(x: np.ndarray, h: np.ndarray, npol: int = 1) -> np.ndarray:
    """u_m = sum_{k=-K}^{K} h_k x_{(m-k) mod n} along the time axis (Sec. III-B)."""
    h = np.asarray(h, dtype=np.complex128)
    T = h.shape[0]
    assert T % 2 == 1, "filter length must be odd (T = 2K + 1)"
    K = (T - 1) // 2
    ax = _time_axis(npol)
    u = np.zeros(x.shape, dtype=np.complex128)
    for k in range(-K, K + 1):
        # np.roll(x, k)[m] = x[(m - k) mod n]
        u = u + h[K + k] * np.roll(x, k, axis=ax)
    return u


def power(u: np.ndarray, npol: int = 1) -> np.ndarray:
    """|u|^2 per time sample; summed over both polarisations for npol = 2."""
    p = u.real * u.real + u.imag * u.imag
    if npol == 2:
        p = p.sum(axis=-1)
    return p


def kerr(u: np.ndarray, c: float, npol: int = 1) -> np.ndarray:
    """sigma(u) = u exp(j c |u|^2) (Sec. III-A, Remark 1); Manakov phase for npol = 2."""
    phi = c * power(u, npol)
    rot = np.exp(1j * phi)
    if npol == 2:
        rot = rot[..., None]
    return u * rot


def ldbp_forward(x: np.ndarray, taps, c, npol: int = 1, return_all: bool = False):
    """Evaluates eq. (model): l steps of circular FIR followed by the Kerr phase.

    ``taps`` is a sequence of l odd-length complex vectors, ``c`` a length-l real
    vector.  Returns y, or (y, ys, us) with ys[i] the input of step i+1 (ys[0] = x,
    ys[l] = y) and us[i] the FIR output of step i+1 when ``return_all``.
    """
    x = np.asarray(x, dtype=np.complex128)
    c = np.asarray(c, dtype=np.float64)
    assert len(taps) == c.shape[0]
    ys = [x]
    us = []
    cur = x
    for i in range(len(taps)):
        u = fir_circular(cur, taps[i], npol)
        cur = kerr(u, c[i], npol)
        us.append(u)
        ys.append(cur)
    if return_all:
        return cur, ys, us
    return cur


def circulant_matrix(h: np.ndarray, n: int) -> np.ndarray:
    """Dense n x n matrix of the circular convolution (Sec. III-B): row m holds h_k in column (m-k) mod n.

    Brute-force construction for tiny n, used to pin ``fir_circular``.
    """
    h = np.asarray(h, dtype=np.complex128)
    K = (h.shape[0] - 1) // 2
    A = np.zeros((n, n), dtype=np.complex128)
    for m in range(n):
        for k in range(-K, K + 1):
            A[m, (m - k) % n] += h[K + k]
    return A


def ldbp_grad(x: np.ndarray, taps, c, gy: np.ndarray, npol: int = 1):
    """Adjoint of ``ldbp_forward`` for a real loss L with dL/dy given as gy.

    Gradient convention for complex z: G = dL/dRe(z) + j dL/dIm(z) (so that a
    real loss changes by Re(conj(G) dz)).  The paper trains with standard tools
    and gives no adjoint; this is the chain rule applied to eq. (model), step by
    step in reverse:

      Kerr  y = u e^{j phi}, phi = c P(u):
            q   = Im(G_y conj(y))            (summed over polarisations for npol = 2)
            dc  = sum q P(u)
            G_u = G_y e^{-j phi} + 2 c q u
      FIR   u_m = sum_k h_k x_{m-k}:
            dh_k = sum_m G_u,m conj(x_{m-k})   (summed over waveforms and polarisations)
            G_x,p = sum_k conj(h_k) G_u,(p+k)

    Returns (gx, gtaps (list), gc).
    """
    c = np.asarray(c, dtype=np.float64)
    y, ys, us = ldbp_forward(x, taps, c, npol, return_all=True)
    G = np.asarray(gy, dtype=np.complex128)
    ax = _time_axis(npol)
    L = len(taps)
    gtaps = [None] * L
    gc = np.zeros(L, dtype=np.float64)
    for i in range(L - 1, -1, -1):
        u = us[i]
        yi = ys[i + 1]
        xin = ys[i]
        P = power(u, npol)
        phi = c[i] * P
        qq = (G * np.conj(yi)).imag
        if npol == 2:
            qq = qq.sum(axis=-1)
        gc[i] = float(np.sum(qq * P))
        rot = np.exp(-1j * phi)
        q2 = 2.0 * c[i] * qq
        if npol == 2:
            rot = rot[..., None]
            q2 = q2[..., None]
        Gu = G * rot + q2 * u
        h = np.asarray(taps[i], dtype=np.complex128)
        K = (h.shape[0] - 1) // 2
        gh = np.zeros(h.shape[0], dtype=np.complex128)
        Gx = np.zeros(Gu.shape, dtype=np.complex128)
        for k in range(-K, K + 1):
            # sum_m G_u,m conj(x_{m-k}); np.roll(xin, k)[m] = xin[m-k]
            gh[K + k] = np.sum(Gu * np.conj(np.roll(xin, k, axis=ax)))
            # G_x,p gets conj(h_k) G_u,(p+k); np.roll(Gu, -k)[p] = Gu[p+k]
            Gx = Gx + np.conj(h[K + k]) * np.roll(Gu, -k, axis=ax)
        gtaps[i] = gh
        G = Gx
    return G, gtaps, gc


def fold_symmetric_grad(gh: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. the symmetric parameterisation h_k = h_{-k} (Sec. III-B): returns (dh_0, dh_1, ..., dh_K)."""
    K = (gh.shape[0] - 1) // 2
    out = np.empty(K + 1, dtype=np.complex128)
    out[0] = gh[K]
    for k in range(1, K + 1):
        out[k] = gh[K + k] + gh[K - k]
    return out
