"""Pins of the oracle's random draws (Algorithm 2, Stage 1, first step)."""
import os

import numpy as np
import pytest

from oracle import rng
from conftest import GOLDEN


def _vectors():
    out = []
    for line in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        out.append([int(v) for v in line.split()])
    return out


@pytest.mark.parametrize("row", _vectors())
def test_mix64_matches_published_splitmix64_stream(row):
    state, outs = row[0], row[1:]
    for o in outs:
        state = (state + rng.GOLDEN) & rng.MASK
        assert rng.mix64(state) == o


def test_h_is_splitmix_stream_from_key():
    # h(seed, st, i) is output i+1 of SplitMix64 started at key(seed, st)
    seed, st = 0xDEADBEEF, 1
    state = rng.key(seed, st)
    for i in range(5):
        state = (state + rng.GOLDEN) & rng.MASK
        assert rng.h(seed, st, i) == rng.mix64(state)


def test_h_array_matches_scalar():
    idx = np.arange(0, 1000, 37, dtype=np.uint64)
    got = rng.h_array(12345, 0, idx)
    want = [rng.h(12345, 0, int(i)) for i in idx]
    assert [int(g) for g in got] == want


def test_signs_balance_and_values():
    d = rng.signs(7, 1 << 16)
    assert set(np.unique(d)) <= {-1.0, 1.0}
    # binomial(65536, 1/2): 5 sigma = 640
    assert abs(d.sum()) < 640
    for t in [0, 1, 99, 65535]:
        assert d[t] == (-1.0 if rng.h(7, 0, t) >> 63 else 1.0)


def test_floyd_small_hand_case():
    # m=5, s=3: iterations j = 2, 3, 4 with r_j = floor(h * (j+1) / 2^64)
    seed = 42
    chosen = []
    for j in range(2, 5):
        r = (rng.h(seed, 1, j) * (j + 1)) >> 64
        chosen.append(j if r in chosen else r)
    assert list(rng.sample_rows(seed, 5, 3)) == sorted(chosen)


def test_floyd_is_subset_sorted_distinct():
    for seed in range(20):
        S = rng.sample_rows(seed, 1000, 64)
        assert len(S) == 64 and len(set(S.tolist())) == 64
        assert np.all(np.diff(S) > 0) and S[0] >= 0 and S[-1] < 1000


def test_floyd_uniform_over_subsets():
    # m=5, s=2: 10 subsets, each with probability 1/10
    counts = {}
    N = 20000
    for seed in range(N):
        key = tuple(rng.sample_rows(seed, 5, 2).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 10
    chi2 = sum((c - N / 10) ** 2 / (N / 10) for c in counts.values())
    assert chi2 < 33.7  # chi-square(9) 99.99th percentile


def test_floyd_full_set_when_s_equals_m():
    assert list(rng.sample_rows(3, 17, 17)) == list(range(17))


def test_floyd_rejects_bad_sizes():
    with pytest.raises(ValueError):
        rng.sample_rows(0, 4, 5)
    with pytest.raises(ValueError):
        rng.sample_rows(0, 4, 0)
