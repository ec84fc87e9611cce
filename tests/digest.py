"""Level digests of canonical characteristic matrices, written in the tests
from the definition in include/ltlf.h (ltlf_result.level_digests), with no
code of the library: canonical rows (the export layout: trace by trace,
positions 0.. as consecutive bits, LSB first in uint64 words) are moved into
the packed layout (per trace t, position k at bit o_t + n_t - 1 - k, a zero
guard bit after each trace, 32-bit words padded to a multiple of 4), hashed
chunk by chunk and summed mod 2^64.

``digest_slow`` restates the same definition with Python integers and loops;
tests pin the vectorised form to it.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

MASK = (1 << 64) - 1
K_GOLD = 0x9E3779B97F4A7C15
K_A = 0xBF58476D1CE4E5B9
K_B = 0x94D049BB133111EB
F1 = 0xFF51AFD7ED558CCD
F2 = 0xC4CEB9FE1A85EC53


def packed_words(lengths: Sequence[int]) -> int:
    nbits = sum(int(n) + 1 for n in lengths)
    return 4 * (((nbits + 31) // 32 + 3) // 4)


def packed_rows(canon: np.ndarray, lengths: Sequence[int]) -> np.ndarray:
    """(n, canonical words) uint64 -> (n, W) uint32 rows of the packed layout."""
    lengths = [int(n) for n in lengths]
    canon = np.ascontiguousarray(canon, dtype=np.uint64)
    n = canon.shape[0]
    npos = sum(lengths)
    W = packed_words(lengths)
    if n == 0:
        return np.zeros((0, W), dtype=np.uint32)
    bits = np.unpackbits(canon.view(np.uint8).reshape(n, -1), axis=1, bitorder="little")[:, :npos]
    out = np.zeros((n, 32 * W), dtype=np.uint8)
    o = g = 0
    for L in lengths:
        out[:, o:o + L] = bits[:, g:g + L][:, ::-1]  # position k -> bit o + L - 1 - k
        o += L + 1
        g += L
    return np.packbits(out, axis=1, bitorder="little").view("<u4").reshape(n, W)


def row_digests(rows: np.ndarray) -> np.ndarray:
    """D(row) for every packed row (uint64 array)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n, W = rows.shape
    if n == 0:
        return np.zeros(0, dtype=np.uint64)
    q = rows.view("<u8").reshape(n, W // 2)
    a, b = q[:, 0::2], q[:, 1::2]
    k = np.arange(1, a.shape[1] + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        m = (a ^ (k * np.uint64(K_GOLD))) * np.uint64(K_A)
        m ^= (b + (m >> np.uint64(31))) * np.uint64(K_B)
        m ^= m >> np.uint64(29)
        x = np.bitwise_xor.reduce(m, axis=1)
        x ^= x >> np.uint64(33)
        x *= np.uint64(F1)
        x ^= x >> np.uint64(33)
        x *= np.uint64(F2)
        x ^= x >> np.uint64(33)
    return x


def level_digest(canon: np.ndarray, lengths: Sequence[int]) -> int:
    """digest(U_c) of a level given as canonical rows."""
    d = row_digests(packed_rows(canon, lengths))
    return int(np.sum(d, dtype=np.uint64)) if len(d) else 0


def digest_slow(canon_rows: Sequence[Sequence[int]], lengths: Sequence[int]) -> int:
    """The same definition with Python integers, one bit at a time."""
    lengths = [int(n) for n in lengths]
    W = packed_words(lengths)
    total = 0
    for row in canon_rows:
        word = [0] * W
        o = g = 0
        for L in lengths:
            for k in range(L):
                gb = g + k
                if (int(row[gb // 64]) >> (gb % 64)) & 1:
                    pb = o + L - 1 - k
                    word[pb // 32] |= 1 << (pb % 32)
            o += L + 1
            g += L
        x = 0
        for c in range(W // 4):
            a = word[4 * c] | (word[4 * c + 1] << 32)
            b = word[4 * c + 2] | (word[4 * c + 3] << 32)
            m = ((a ^ ((c + 1) * K_GOLD & MASK)) * K_A) & MASK
            m ^= ((b + (m >> 31)) * K_B) & MASK
            m ^= m >> 29
            x ^= m
        x ^= x >> 33
        x = (x * F1) & MASK
        x ^= x >> 33
        x = (x * F2) & MASK
        x ^= x >> 33
        total = (total + x) & MASK
    return total
