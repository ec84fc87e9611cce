"""CPU pins of the tests' level-digest helper (tests/digest.py): the packed
layout on a hand-worked example, the vectorised digest against its
one-bit-at-a-time restatement, and the properties a set fingerprint needs."""
from __future__ import annotations

import numpy as np

from tests import digest


def test_packed_layout_hand_example():
    # trace 0 (length 3): positions 0, 1, 2 = 1, 0, 0; trace 1 (length 2): 0, 1
    # canonical bits: 1 0 0 | 0 1  -> word 0b10001
    canon = np.array([[0b10001]], dtype=np.uint64)
    rows = digest.packed_rows(canon, [3, 2])
    # trace 0 at bits 0..2 reversed (position 0 at bit 2), guard bit 3;
    # trace 1 at bits 4..5 (position 0 at bit 5, position 1 at bit 4), guard 6
    assert rows.shape == (1, 4)
    assert rows[0].tolist() == [(1 << 2) | (1 << 4), 0, 0, 0]


def test_packed_width_rounds_to_whole_chunks():
    assert digest.packed_words([3, 2]) == 4
    assert digest.packed_words([31]) == 4          # 32 bits
    assert digest.packed_words([32]) == 4          # 33 bits -> 2 words -> 4
    assert digest.packed_words([64] * 2) == 8      # 130 bits -> 5 words -> 8


def test_vectorised_digest_equals_slow_restatement():
    rng = np.random.default_rng(11)
    for trial in range(6):
        lengths = [int(x) for x in rng.integers(1, 70, size=int(rng.integers(1, 9)))]
        npos = sum(lengths)
        cw = (npos + 63) // 64
        canon = rng.integers(0, 1 << 63, size=(5, cw), dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=(5, cw), dtype=np.uint64)
        if npos % 64:
            canon[:, -1] &= np.uint64((1 << (npos % 64)) - 1)
        got = digest.level_digest(canon, lengths)
        want = digest.digest_slow(canon.tolist(), lengths)
        assert got == want, (trial, lengths)


def test_digest_is_a_set_fingerprint():
    rng = np.random.default_rng(5)
    lengths = [7, 12, 3, 30]
    canon = rng.integers(0, 1 << 52, size=(40, 1), dtype=np.uint64)
    d = digest.level_digest(canon, lengths)
    assert digest.level_digest(canon[::-1], lengths) == d          # order does not matter
    assert digest.level_digest(canon[1:], lengths) != d            # a missing CM shows
    flip = canon.copy()
    flip[3, 0] ^= np.uint64(1 << 40)
    assert digest.level_digest(flip, lengths) != d                 # one changed bit shows
    assert digest.level_digest(canon[:0], lengths) == 0            # empty level
