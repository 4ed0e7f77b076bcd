"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and lays out arrays.  It holds none of
the method's arithmetic (no filtering, no split-step, no pulse shaping): every
random quantity the method consumes -- symbol indices, amplifier noise, training
powers, tap perturbations -- is drawn here and handed to both the oracle and the
HIP path as an explicit input, so the two sides never share code.

All draws use NumPy's PCG64 generator keyed by an integer seed and a small
integer "stream" tag, so that e.g. the symbols and the noise of one workload are
independent but reproducible.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "qam16_indices",
    "complex_normal",
    "uniform_choice",
    "log_uniform_lengths",
    "random_taps",
    "random_real",
]


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """A PCG64 generator for (seed, stream); distinct streams are independent."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def qam16_indices(seed: int, shape, stream: int = 1) -> np.ndarray:
    """I.i.d. uniform symbol indices in 0..15 (int32)."""
    return rng(seed, stream).integers(0, 16, size=shape, dtype=np.int32)


def complex_normal(seed: int, shape, stream: int = 2, dtype=np.complex128) -> np.ndarray:
    """I.i.d. circularly-symmetric complex Gaussian samples with E|w|^2 = 1."""
    g = rng(seed, stream)
    re = g.standard_normal(size=shape)
    im = g.standard_normal(size=shape)
    return ((re + 1j * im) * np.sqrt(0.5)).astype(dtype)


def uniform_choice(seed: int, values, size, stream: int = 3) -> np.ndarray:
    """Draws uniformly from a finite set (e.g. the training power set)."""
    values = np.asarray(values)
    return values[rng(seed, stream).integers(0, len(values), size=size)]


def log_uniform_lengths(seed: int, count: int, lo: int, hi: int, stream: int = 4) -> np.ndarray:
    """Raw log-uniform draws in [lo, hi] (float64, before any rounding rule)."""
    u = rng(seed, stream).uniform(np.log(lo), np.log(hi), size=count)
    return np.exp(u)


def random_taps(seed: int, ntaps, scale: float = 1.0, stream: int = 5) -> list[np.ndarray]:
    """One complex CN(0, scale^2) tap vector per entry of ``ntaps``."""
    g = rng(seed, stream)
    out = []
    for t in ntaps:
        v = (g.standard_normal(int(t)) + 1j * g.standard_normal(int(t))) * (scale * np.sqrt(0.5))
        out.append(v)
    return out


def random_real(seed: int, shape, lo: float = -1.0, hi: float = 1.0, stream: int = 6) -> np.ndarray:
    """Uniform reals in [lo, hi)."""
    return rng(seed, stream).uniform(lo, hi, size=shape)
