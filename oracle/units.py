"""Physical constants and unit conversions (Table I; Sec. IV-A).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

All quantities are SI: metres, seconds, watts, hertz.
  alpha  power attenuation coefficient [1/m]; the field decays as exp(-alpha z / 2) (eq. nlse)
  beta2  group-velocity dispersion [s^2/m]
  gamma  Kerr coefficient [1/(W m)]
"""
from __future__ import annotations

import math

PLANCK = 6.626e-34          # Table I, h [J s]
NU_S = 1.946e14             # Table I, optical carrier frequency [Hz]


def alpha_from_db_per_km(db_per_km: float) -> float:
    """Table I gives alpha = 0.2 dB/km (power); returns the natural-log coefficient in 1/m."""
    return db_per_km * math.log(10.0) / 10.0 / 1e3


def beta2_from_ps2_per_km(ps2_per_km: float) -> float:
    """Table I gives beta2 = -21.683 ps^2/km; returns s^2/m."""
    return ps2_per_km * 1e-24 / 1e3


def gamma_from_per_w_per_km(g: float) -> float:
    """Table I gives gamma = 1.3 1/(W km); returns 1/(W m)."""
    return g / 1e3


def dbm_to_watt(p_dbm: float) -> float:
    return 10.0 ** ((p_dbm - 30.0) / 10.0)


def db_to_lin(x_db: float) -> float:
    return 10.0 ** (x_db / 10.0)


def lin_to_db(x: float) -> float:
    return 10.0 * math.log10(x)


def l_eff(z: float, alpha: float) -> float:
    """Effective nonlinear length (1 - e^{-alpha z}) / alpha (Sec. III-A); equals z for alpha = 0."""
    if alpha == 0.0:
        return float(z)
    return (1.0 - math.exp(-alpha * z)) / alpha


def ase_variance_per_sample(alpha: float, span_len: float, nf_db: float, fs: float,
                            nu_s: float = NU_S, h: float = PLANCK) -> float:
    """Per-sample variance of the complex ASE noise added by one EDFA (Sec. IV-A).

    The amplifier adds white Gaussian noise of power spectral density
    (e^{alpha L_sp} - 1) h nu_s n_sp with n_sp = NF / (2 (1 - e^{-alpha L_sp})).
    Sampled at rate fs, white noise of that PSD has per-sample variance PSD * fs.
    """
    nf = db_to_lin(nf_db)
    n_sp = nf / (2.0 * (1.0 - math.exp(-alpha * span_len)))
    psd = (math.exp(alpha * span_len) - 1.0) * h * nu_s * n_sp
    return psd * fs


def t_cd(beta2: float, delta_f: float, length: float, fs: float) -> float:
    """CD memory in samples, eq. required_length, with |beta2| (the printed form is negative for beta2 < 0)."""
    return 2.0 * math.pi * abs(beta2) * delta_f * length * fs
