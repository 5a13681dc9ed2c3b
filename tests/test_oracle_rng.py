"""Pins of the reference's counter-based generator (Philox4x32-10)."""
import os

import numpy as np
from scipy import stats

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors(oracle_mod):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle_mod.philox(ctr, key).tolist() == out


def test_philox_uniform_and_uncorrelated(oracle_mod):
    # 20k counters -> 80k words; chi-square on 64 bins of the top bits and
    # lag-1 serial correlation of consecutive words
    n = 20000
    words = np.concatenate([oracle_mod.philox([i, 7, 3, 0x10], [12345, 678]) for i in range(n)])
    bins = np.bincount(words >> np.uint32(26), minlength=64)
    chi2, p = stats.chisquare(bins)
    assert p > 1e-4, (chi2, p)
    u = (words.astype(np.float64) + 0.5) / 2.0 ** 32
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 4.0 / np.sqrt(len(u))
    # counter words other than word 0 also decorrelate the stream
    a = np.array([oracle_mod.philox([5, j, 0, 0], [1, 2])[0] for j in range(4000)], dtype=np.float64)
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 4.0 / np.sqrt(len(a))


def test_philox_key_sensitivity(oracle_mod):
    a = oracle_mod.philox([1, 2, 3, 4], [5, 6])
    b = oracle_mod.philox([1, 2, 3, 4], [5, 7])
    c = oracle_mod.philox([1, 2, 3, 5], [5, 6])
    flips = sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b))
    flips2 = sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, c))
    # avalanche: about half of 128 bits flip
    assert 40 < flips < 88 and 40 < flips2 < 88
