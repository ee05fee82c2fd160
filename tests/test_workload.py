"""The seeded input generators: their streams have the distributions their
docstrings state (checked against exact formulas on small cases)."""

import numpy as np

from paper_1712_09624_amd import workload as W


def test_five_tuple_layout():
    k = W.five_tuples(4096, 3).view(np.uint32).reshape(-1, 4)
    assert set(np.unique(k[:, 3] & 0xFF)) == {6, 17}
    assert not (k[:, 3] >> 8).any()  # three zero bytes


def test_keys_at_load_rounds_half_up():
    assert W.keys_at_load(14, 0.8) == 104858  # 0.8 * 131072 = 104857.6
    assert W.keys_at_load(1, 0.5) == 8


def test_many_tables_ranges():
    c = W.many_tables(4000, 5)
    assert c["log2_buckets"].min() == 10 and c["log2_buckets"].max() == 18
    assert set(np.unique(c["log2_buckets"])) == set(range(10, 19))
    assert (c["load"] >= 0.6).all() and (c["load"] < 0.95).all()
    assert c["batch"].min() >= 32 and c["batch"].max() <= 4096
    assert (c["neg_rate"] >= 0).all() and (c["neg_rate"] < 1).all()
    # the exponent is uniform: each of the 9 values within 5 sigma of 4000/9
    counts = np.bincount(c["log2_buckets"])[10:]
    assert (np.abs(counts - 4000 / 9) < 5 * np.sqrt(4000 / 9)).all()


def test_zipf_ranks_follow_the_power_law():
    # on a universe of 1000 ranks the empirical frequency of each of the
    # first ranks matches the continuous approximation's mass of [r+1, r+2)
    # exactly (within sampling error), and the rank ratio follows x^-s
    n, N, s = 2_000_000, 1000, 1.1
    r = W.zipf_ranks(n, N, s, 7, 11)
    assert r.min() >= 0 and r.max() < N
    a = 1 - s
    mass = lambda x: (x ** a - 1) / ((N + 1) ** a - 1)  # P(X < x)
    for rank in (0, 1, 2, 9, 99):
        p = mass(rank + 2) - mass(rank + 1)
        f = (r == rank).mean()
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / n), (rank, f, p)


def test_poisson_arrivals_mean_gap():
    t = W.poisson_arrivals(200_000, 1e5, 3, 4)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert (gaps > 0).all()
    assert abs(gaps.mean() - 1e-5) < 5 * 1e-5 / np.sqrt(len(gaps))
    # exponential: the share of gaps above the mean is e^-1
    assert abs((gaps > 1e-5).mean() - np.exp(-1)) < 0.005
