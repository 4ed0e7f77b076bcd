"""Distribution pins for the oracle's Philox4x32-10 + Box-Muller noise generator."""
import numpy as np

from oracle import philox as P


def test_words_uniform():
    w = P.words(1 << 15, seed=123, stream=7)
    b = (w >> np.uint64(24)).astype(np.int64).reshape(-1)  # top byte of every word
    counts = np.bincount(b, minlength=256)
    exp = b.size / 256
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < 255 + 5 * np.sqrt(2 * 255)


def test_counter_changes_every_word():
    w = P.words(4, seed=1, stream=0)
    assert len({int(x) for x in w.reshape(-1)}) == 16


def test_normal_moments_and_tail():
    z = P.complex_normal(1 << 18, seed=5, stream=3)
    assert abs(np.mean(z)) < 0.01
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.01
    assert abs(np.mean(z * z)) < 0.01  # circular symmetry
    assert abs(np.var(z.real) - 0.5) < 0.01
    # P(|z|^2 > 4) = e^{-4} for CN(0,1)
    assert abs(np.mean(np.abs(z) ** 2 > 4.0) - np.exp(-4.0)) < 0.002


def test_streams_and_keys_independent():
    a = P.complex_normal(1 << 16, seed=5, stream=3)
    b = P.complex_normal(1 << 16, seed=5, stream=4)
    c = P.complex_normal(1 << 16, seed=6, stream=3)
    for u, v in ((a, b), (a, c)):
        assert abs(np.mean(u * np.conj(v))) < 0.02
