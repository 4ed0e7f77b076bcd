"""Counter-based Philox4x32-10 and a Box-Muller complex normal (Salmon, Moraes, Dror, Shaw, SC'11).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Used to model the amplifier noise that the channel simulator draws on the GPU
during training (Sec. IV-A: each EDFA adds white Gaussian noise).  Written from
the published definition of the Philox-4x32 bijection: ten rounds, each
multiplying words 0 and 2 by the round multipliers, swapping and XOR-ing the
high halves with the remaining words and the round key, with the key bumped by
the Weyl constants between rounds.

Stream layout (shared convention with the device generator): complex normal
number i of a call with key (seed) and 64-bit stream id uses counter
(i//2 mod 2^32, i//2 >> 32, stream mod 2^32, stream >> 32); output words w0,w1
feed sample 2p and w2,w3 sample 2p+1.  Each word pair (a, b) maps to
u_a = (a + 0.5) 2^-32, u_b = (b + 0.5) 2^-32 and
w = sqrt(-ln u_a) (cos 2 pi u_b + j sin 2 pi u_b), so E|w|^2 = 1.

Pins (tests/test_oracle_philox.py): the three published known-answer vectors
of the Random123 test set (tests/golden/philox_kat.json), which fix the round
function, both multipliers and the key schedule; the Weyl constants recomputed
from their definition (the first 32 fractional bits of the golden ratio and of
sqrt(3) - 1); the counter layout of words(); distribution tests (uniformity of
the words, moments and tail of the normals, independence of streams).  The
device generator is held to bit equality with this one.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def _mulhilo(a, b):
    p = a.astype(np.uint64) * np.uint64(b)
    return (p >> np.uint64(32)).astype(np.uint64), (p & np.uint64(MASK)).astype(np.uint64)


def philox4x32_10(ctr: np.ndarray, key: tuple[int, int]) -> np.ndarray:
    """ctr: uint64 array [..., 4] holding 32-bit words; returns the 4 output words (uint64 holding uint32)."""
    c = [ctr[..., i].astype(np.uint64) & np.uint64(MASK) for i in range(4)]
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for r in range(10):
        hi0, lo0 = _mulhilo(c[0], M0)
        hi1, lo1 = _mulhilo(c[2], M1)
        c = [
            (hi1 ^ c[1] ^ np.uint64(k0)) & np.uint64(MASK),
            lo1,
            (hi0 ^ c[3] ^ np.uint64(k1)) & np.uint64(MASK),
            lo0,
        ]
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return np.stack(c, axis=-1)


def words(count_pairs: int, seed: int, stream: int) -> np.ndarray:
    """Raw output words for counters p = 0..count_pairs-1: shape [count_pairs, 4]."""
    p = np.arange(count_pairs, dtype=np.uint64)
    ctr = np.zeros((count_pairs, 4), dtype=np.uint64)
    ctr[:, 0] = p & np.uint64(MASK)
    ctr[:, 1] = p >> np.uint64(32)
    ctr[:, 2] = np.uint64(stream & MASK)
    ctr[:, 3] = np.uint64((stream >> 32) & MASK)
    key = (seed & MASK, (seed >> 32) & MASK)
    return philox4x32_10(ctr, key)


def complex_normal(count: int, seed: int, stream: int) -> np.ndarray:
    """count CN(0, 1) samples of the stream (E|w|^2 = 1)."""
    pairs = (count + 1) // 2
    w = words(pairs, seed, stream).astype(np.float64)
    ua = (w[:, [0, 2]] + 0.5) * 2.0 ** -32
    ub = (w[:, [1, 3]] + 0.5) * 2.0 ** -32
    r = np.sqrt(-np.log(ua))
    z = r * (np.cos(2.0 * np.pi * ub) + 1j * np.sin(2.0 * np.pi * ub))
    return z.reshape(-1)[:count]
