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


def _kat():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")) as fh:
        return json.load(fh)


def test_known_answer_vectors():
    """The published Random123 known-answer words (golden/philox_kat.json): pins the round function,
    both multipliers and the key schedule, which the distribution tests above cannot tell apart."""
    for v in _kat()["vectors"]:
        ctr = np.array([int(w, 16) for w in v["ctr"]], dtype=np.uint64)
        key = tuple(int(w, 16) for w in v["key"])
        out = P.philox4x32_10(ctr, key)
        assert [int(w) for w in out] == [int(w, 16) for w in v["out"]]


def test_weyl_constants_from_their_definition():
    """W0 and W1 are the first 32 fractional bits of the golden ratio and of sqrt(3) - 1 (exact
    integer arithmetic: floor(2^32 x) for x = (sqrt(5) - 1) / 2 and sqrt(3) - 1)."""
    from math import isqrt
    # floor(2^32 (sqrt(5) - 1) / 2) = floor((sqrt(5 * 2^64) - 2^32) / 2)
    w0 = (isqrt(5 << 64) - (1 << 32)) // 2
    w1 = isqrt(3 << 64) - (1 << 32)
    assert P.W0 == w0 and P.W1 == w1


def test_words_layout_matches_bijection():
    """words() feeds counter (p lo, p hi, stream lo, stream hi) and key (seed lo, seed hi)."""
    seed, stream = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    w = P.words(3, seed, stream)
    for p in range(3):
        ctr = np.array([p, 0, stream & 0xFFFFFFFF, stream >> 32], dtype=np.uint64)
        ref = P.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        assert np.array_equal(w[p], ref)
