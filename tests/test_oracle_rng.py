"""Pins for the oracle's Philox4x32-10 generator and stream derivation.

The reference here is an independent pure-Python Philox written from the
SC'11 description (Salmon et al., "Parallel random numbers: as easy as 1, 2,
3"), itself checked against the published known-answer vectors."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")
M = 0xFFFFFFFF


def py_philox(ctr, key, rounds=10):
    c = [int(x) & M for x in ctr]
    k = [int(x) & M for x in key]
    for _ in range(rounds):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & M, p1 & M, ((p0 >> 32) ^ c[3] ^ k[1]) & M, p0 & M]
        k = [(k[0] + 0x9E3779B9) & M, (k[1] + 0xBB67AE85) & M]
    return c


def test_python_reference_matches_published_vectors():
    for case in json.load(open(GOLD))["cases"]:
        out = py_philox([int(x, 16) for x in case["ctr"]], [int(x, 16) for x in case["key"]])
        assert out == [int(x, 16) for x in case["out"]]


def test_oracle_philox_matches_python(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(2000):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64)
        key = rng.integers(0, 2**32, 2, dtype=np.uint64)
        assert list(oracle_lib.philox(ctr, key)) == py_philox(ctr, key)


def test_uniform_bit_mapping(oracle_lib):
    """u = (w0 * 2^21 + (w1 >> 11)) * 2^-53, counter (block, stream)."""
    seed = 0x0123456789ABCDEF
    for block in (0, 1, 7, 2**31 + 5):
        stream = [11, 22, (3 << 8) | 1]
        w = py_philox([block] + stream, [seed & M, seed >> 32])
        want = ((w[0] << 21) + (w[1] >> 11)) / 2.0**53
        assert oracle_lib.uniform_at(seed, stream, block) == want


def test_uniform_statistics(oracle_lib):
    """Equidistribution (chi^2 over 64 cells) and lag-1 independence."""
    u = np.array([oracle_lib.uniform_at(0, [i, 0, 1], b) for i in range(200) for b in range(100)])
    assert u.min() >= 0.0 and u.max() < 1.0
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = len(u) / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 63 + 5 * np.sqrt(2 * 63)
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / np.sqrt(len(u))


def test_child_streams_are_distinct_and_tagged(oracle_lib):
    seen = set()
    for p in range(50):
        parent = [p, 0, 1]
        for blk in range(20):
            ch = oracle_lib.child_stream(7, parent, blk)
            assert ch[2] & 0x80000000
            w = py_philox([blk] + parent, [(7 & M) ^ 0x9E3779B9, 0])
            assert list(ch) == [w[0], w[1], w[2] | 0x80000000]
            seen.add(tuple(ch))
    assert len(seen) == 50 * 20
